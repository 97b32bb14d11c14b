// Coarsest-level block preconditioner (FP64): numeric smoothed-aggregation
// setup from host-built gather lists, the AMG V-cycle on d right-hand sides
// (vectors stored [row][component]), and the pressure / velocity split of the
// block-triangular Stokes preconditioner
//   y = -g / S_T,   x = AMG(f - C y).
// The V-cycle is evaluated with B = A P (formed by the Galerkin setup): the
// restricted residual after pre-smoothing is P^T r - B^T x, and prolongation with
// the first post-sweep is x + P x_c + w D^{-1} (r - A x - B x_c) (4 launches per
// level).  The levels from the first one with at most coarse_amg_explicit rows
// down are applied as the explicit matrix of their V-cycle, formed at setup by
// running the V-cycle on the identity columns (column-block kernels k_cols_*).
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

// D^{-1} and the power-iteration start vector v_i = frac(i * 2654435761 / 2^32) - 1/2
__global__ void k_amg_diag(int n, const int32_t *diag, const double *val, double *dinv, double *v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    dinv[i] = 1.0 / val[diag[i]];
    const uint64_t h = ((uint64_t)i * 2654435761ull) % 4294967296ull;
    v[i] = (double)h / 4294967296.0 - 0.5;
  }
}

// One power-iteration step for lambda ~ rho(D^{-1} A): vout = D^{-1} A vin / |vin|,
// with |vin|^2 the sum of the nin partial sums pin (nin == 0: no scaling; every
// block adds them in the same order), and this block's share of |vout|^2 in
// pout[blockIdx.x].  G lanes per row.  k_amg_power_finish writes
// lam_out = safety * |vout| after the last step.
template <int G>
__global__ void __launch_bounds__(kBlock) k_amg_power(int n, const int32_t *rp, const int32_t *ci, const double *val,
                                                       const double *dinv, const double *vin, const double *pin,
                                                       int nin, double *vout, double *pout) {
  __shared__ double red[16];
  __shared__ double scs;
  double sc = 1.0;
  if (nin > 0) {
    if (threadIdx.x < kWave) {
      double t = 0;
      for (int b = threadIdx.x; b < nin; b += kWave) t += pin[b];
      t = wave_sum(t);
      if (threadIdx.x == 0) scs = 1.0 / sqrt(t);
    }
    __syncthreads();
    sc = scs;
  }
  const int lane = threadIdx.x % G;
  const int64_t ngroups = (int64_t)gridDim.x * (blockDim.x / G);
  double acc = 0;
  for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G; i < n; i += ngroups) {
    double t = 0;
    for (int e = rp[i] + lane; e < rp[i + 1]; e += G) t += val[e] * vin[ci[e]];
    t = group_sum<G>(t);
    if (lane == 0) {
      t *= sc * dinv[i];
      vout[i] = t;
      acc += t * t;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) pout[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_amg_power_finish(int G, const double *partial, double *lam_out,
                                                              double safety) {
  __shared__ double tot[1];
  reduce_partials(partial, G, 1, tot);
  if (threadIdx.x == 0) lam_out[0] = safety * sqrt(tot[0]);
}

// second smoothing step: P = P_1 - (omega / lambda) D^{-1} B_1 with B_1 = A P_1
// on the final pattern (src: the entry's P_1 entry, or -1)
__global__ void k_amg_p2(int64_t npe, const int32_t *src, const int32_t *prow, const double *p1, const double *b1,
                         const double *dinv, const double *lam, double *pval) {
  const double w = kAmgOmegaSA / lam[0];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npe; e += (int64_t)gridDim.x * blockDim.x)
    pval[e] = (src[e] >= 0 ? p1[src[e]] : 0.0) - w * dinv[prow[e]] * b1[e];
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

// coarsest level: dense inverse of the (small, SPD) CSR matrix by Gauss-Jordan
// elimination without pivoting (the pivots of an SPD matrix are positive), the
// matrix resident in LDS, one block of 1024 threads; n <= kAmgCoarsest.
__global__ void __launch_bounds__(1024) k_amg_coarsest_lds(int n, const int32_t *rp, const int32_t *ci,
                                                            const double *val, double *Ainv, int *err) {
  extern __shared__ double lds[];
  double *M = lds, *colk = lds + n * n, *rowk = colk + n;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) M[i] = 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int e = rp[i]; e < rp[i + 1]; ++e) M[i * n + ci[e]] = val[e];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = M[k * n + k];
    if (!(piv > 0)) {
      if (threadIdx.x == 0) bad = 1;
      break;  // uniform: every thread reads the same pivot
    }
    const double ip = 1.0 / piv;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      colk[i] = M[i * n + k];
      rowk[i] = M[k * n + i] * ip;
    }
    __syncthreads();
    // M_ij -= M_ik M_kj / piv (i, j != k); row k scaled by 1/piv; column k = -M_ik / piv; M_kk = 1/piv
    for (int o = threadIdx.x; o < n * n; o += blockDim.x) {
      const int i = o / n, j = o % n;
      double v;
      if (i == k) v = (j == k) ? ip : rowk[j];
      else if (j == k) v = -colk[i] * ip;
      else v = M[o] - colk[i] * rowk[j];
      M[o] = v;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) Ainv[i] = M[i];
  if (threadIdx.x == 0 && bad) atomicMax(err, 1);
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
                         double *rhs, double *z, const int *skip) {
  if (skip && *skip) return;
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

// Damped-Jacobi sweep xout = xin + w D^{-1} (r - A xin), G lanes per row, all d
// (<= 3) components at once; xin == null means xin = w D^{-1} r (a first sweep
// from zero folded in), so one launch gives two sweeps.
template <int G>
__global__ void __launch_bounds__(kBlock) k_amg_rows(int n, int d, const int32_t *rp, const int32_t *ci,
                                                      const double *val, const double *dinv, const double *lam,
                                                      const double *r, const double *xin, double *xout,
                                                      const int *skip) {
  if (skip && *skip) return;
  const double w = kAmgOmegaJac / lam[0];
  const int lane = threadIdx.x % G;
  const int64_t ngroups = (int64_t)gridDim.x * (blockDim.x / G);
  for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G; i < n; i += ngroups) {
    double t0 = 0, t1 = 0, t2 = 0;
    for (int e = rp[i] + lane; e < rp[i + 1]; e += G) {
      const int j = ci[e];
      const double a = val[e];
      double x0, x1 = 0, x2 = 0;
      if (xin) {
        const double *xj = xin + (int64_t)j * d;
        x0 = xj[0];
        if (d > 1) x1 = xj[1];
        if (d > 2) x2 = xj[2];
      } else {
        const double sc = w * dinv[j];
        const double *rj = r + (int64_t)j * d;
        x0 = sc * rj[0];
        if (d > 1) x1 = sc * rj[1];
        if (d > 2) x2 = sc * rj[2];
      }
      t0 += a * x0;
      t1 += a * x1;
      t2 += a * x2;
    }
    t0 = group_sum<G>(t0);
    t1 = group_sum<G>(t1);
    t2 = group_sum<G>(t2);
    if (lane != 0) continue;
    const double si = w * dinv[i];
    double y[3] = {0, 0, 0}, q[3] = {t0, t1, t2};
    for (int c = 0; c < d; ++c) {
      const double rc = r[i * d + c];
      y[c] = xin ? xin[i * d + c] : si * rc;
      q[c] = rc - q[c];
    }
    for (int c = 0; c < d; ++c) xout[i * d + c] = y[c] + si * q[c];
  }
}

// dst[k] = src[idx[k]] (values of a matrix in the order of its transpose)
__global__ void __launch_bounds__(kBlock) k_amg_gather(int64_t n, const int32_t *idx, const double *src,
                                                        double *dst) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src[idx[k]];
}

// s += sign * sum over k in [beg, end) of v[k] * x(row[k]), the wavefront's lanes
// taking every 64th entry, four entries in flight per lane.  With scale != null
// the vector is x(i) = w scale[i] y[i] (a sweep from zero), else x(i) = y[i].
template <int SIGN>
__device__ inline void wave_gather(int beg, int end, const int32_t *row, const double *v, const double *y,
                                   const double *scale, double w, int d, double &s0, double &s1, double &s2) {
  const int lane = threadIdx.x % kWave;
  for (int k = beg + lane; k < end; k += 4 * kWave) {
    int ii[4];
    double vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k + u * kWave;
      const bool in = kk < end;
      ii[u] = in ? row[kk] : 0;
      vv[u] = in ? v[kk] : 0.0;
    }
    if (scale) {
#pragma unroll
      for (int u = 0; u < 4; ++u) vv[u] *= w * scale[ii[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double *yi = y + (int64_t)ii[u] * d;
      s0 += SIGN * vv[u] * yi[0];
      if (d > 1) s1 += SIGN * vv[u] * yi[1];
      if (d > 2) s2 += SIGN * vv[u] * yi[2];
    }
  }
}

// rc = P^T r - B^T x with B = A P: since A is symmetric, B^T x = P^T A x, so this
// is the restriction of the residual r - A x after pre-smoothing, with no pass
// that forms that residual.  x == null stands for x = w D^{-1} r (one sweep from
// zero).  One wavefront per coarse row; lanes split the P^T and B^T entries.
__global__ void __launch_bounds__(kBlock) k_amg_restrict(int nc, int d, const int32_t *ptp, const int32_t *pti,
                                                          const double *ptval, const int32_t *btp,
                                                          const int32_t *bti, const double *btval,
                                                          const double *dinv, const double *lam, const double *r,
                                                          const double *x, double *rc, const int *skip) {
  if (skip && *skip) return;
  const double w = kAmgOmegaJac / lam[0];
  const int lane = threadIdx.x % kWave;
  const int64_t nwave = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave; I < nc; I += nwave) {
    double s0 = 0, s1 = 0, s2 = 0;
    wave_gather<1>(ptp[I], ptp[I + 1], pti, ptval, r, nullptr, 0.0, d, s0, s1, s2);
    wave_gather<-1>(btp[I], btp[I + 1], bti, btval, x ? x : r, x ? nullptr : dinv, w, d, s0, s1, s2);
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

// Prolongation and the first post-smoothing sweep in one pass: with
// c = xin + P xc, xout = c + w D^{-1} (r - A c) is evaluated as
// xin + P xc + w D^{-1} (r - A xin - B xc) (B = A P), so no row needs the
// corrected values of its neighbours.  xin == null stands for xin = w D^{-1} r.
// G lanes per row; xout must not alias xin.
template <int G>
__global__ void __launch_bounds__(kBlock) k_amg_prolong_sweep(int n, int d, const int32_t *rp, const int32_t *ci,
                                                               const double *val, const double *dinv,
                                                               const double *lam, const int32_t *prp,
                                                               const int32_t *pci, const double *pval,
                                                               const int32_t *brp, const int32_t *bci,
                                                               const double *bval, const double *xc,
                                                               const double *r, const double *xin, double *xout,
                                                               const int *skip) {
  if (skip && *skip) return;
  const double w = kAmgOmegaJac / lam[0];
  const int lane = threadIdx.x % G;
  const int64_t ngroups = (int64_t)gridDim.x * (blockDim.x / G);
  for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G; i < n; i += ngroups) {
    double q0 = 0, q1 = 0, q2 = 0;  // (A xin + B xc)_i
    double p0 = 0, p1 = 0, p2 = 0;  // (P xc)_i
    for (int e = rp[i] + lane; e < rp[i + 1]; e += G) {
      const int j = ci[e];
      double a = val[e];
      const double *xj = xin ? xin + (int64_t)j * d : r + (int64_t)j * d;
      if (!xin) a *= w * dinv[j];
      q0 += a * xj[0];
      if (d > 1) q1 += a * xj[1];
      if (d > 2) q2 += a * xj[2];
    }
    for (int e = brp[i] + lane; e < brp[i + 1]; e += G) {
      const double bv = bval[e];
      const double *xj = xc + (int64_t)bci[e] * d;
      q0 += bv * xj[0];
      if (d > 1) q1 += bv * xj[1];
      if (d > 2) q2 += bv * xj[2];
    }
    for (int e = prp[i] + lane; e < prp[i + 1]; e += G) {
      const double pv = pval[e];
      const double *xj = xc + (int64_t)pci[e] * d;
      p0 += pv * xj[0];
      if (d > 1) p1 += pv * xj[1];
      if (d > 2) p2 += pv * xj[2];
    }
    q0 = group_sum<G>(q0);
    q1 = group_sum<G>(q1);
    q2 = group_sum<G>(q2);
    p0 = group_sum<G>(p0);
    p1 = group_sum<G>(p1);
    p2 = group_sum<G>(p2);
    if (lane != 0) continue;
    const double si = w * dinv[i], q[3] = {q0, q1, q2}, pp[3] = {p0, p1, p2};
    for (int c = 0; c < d; ++c) {
      const double rc = r[i * d + c];
      const double y = xin ? xin[i * d + c] : si * rc;
      xout[i * d + c] = y + pp[c] + si * (rc - q[c]);
    }
  }
}

// x = Ainv r (dense, row-major n x n): one block per row, every thread taking
// every 256th entry, two in flight; waves combined through LDS
__global__ void __launch_bounds__(kBlock) k_amg_dense(int n, int d, const double *Ainv, const double *r,
                                                       double *x, const int *skip) {
  if (skip && *skip) return;
  __shared__ double red[3][kBlock / kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const double *row = Ainv + i * n;
    double s0 = 0, s1 = 0, s2 = 0;
    int j = threadIdx.x;
    for (; j + kBlock < n; j += 2 * kBlock) {
      const double a0 = row[j], a1 = row[j + kBlock];
      const double *r0 = r + (int64_t)j * d, *r1 = r + (int64_t)(j + kBlock) * d;
      s0 += a0 * r0[0] + a1 * r1[0];
      if (d > 1) s1 += a0 * r0[1] + a1 * r1[1];
      if (d > 2) s2 += a0 * r0[2] + a1 * r1[2];
    }
    if (j < n) {
      const double a0 = row[j];
      const double *r0 = r + (int64_t)j * d;
      s0 += a0 * r0[0];
      if (d > 1) s1 += a0 * r0[1];
      if (d > 2) s2 += a0 * r0[2];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      red[0][wid] = s0;
      red[1][wid] = s1;
      red[2][wid] = s2;
    }
    __syncthreads();
    if (threadIdx.x < d) {
      double t = 0;
      for (int w = 0; w < kBlock / kWave; ++w) t += red[threadIdx.x][w];
      x[i * d + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// ---- explicit V-cycle operator: the V-cycle of a small level applied to the m
// columns of the identity, the same steps as the vector path on [n][m] blocks
// (row-major, one thread per entry), so that M[i][c] = (V e_c)_i.

__global__ void __launch_bounds__(kBlock) k_cols_identity(int64_t n, double *R) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n * n; o += (int64_t)gridDim.x * blockDim.x)
    R[o] = (o / n == o % n) ? 1.0 : 0.0;
}

// Y = X + w D^{-1} (R - A X); X == null stands for X = w D^{-1} R (two sweeps
// from zero in one pass); with half, Y = w D^{-1} R (one sweep from zero).
// These column-block kernels loop over their entries with a grid stride.
__global__ void __launch_bounds__(kBlock) k_cols_sweep(int n, int m, const int32_t *rp, const int32_t *ci,
                                                        const double *val, const double *dinv, const double *lam,
                                                        const double *R, const double *X, double *Y, int half) {
  const double w = kAmgOmegaJac / lam[0];
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < (int64_t)n * m;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / m), c = (int)(o % m);
    const double si = w * dinv[i];
    if (half) {
      Y[o] = si * R[o];
      continue;
    }
    double q = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int64_t jc = (int64_t)ci[e] * m + c;
      q += val[e] * (X ? X[jc] : w * dinv[ci[e]] * R[jc]);
    }
    Y[o] = (X ? X[o] : si * R[o]) + si * (R[o] - q);
  }
}

// T = R - A X
__global__ void __launch_bounds__(kBlock) k_cols_resid(int n, int m, const int32_t *rp, const int32_t *ci,
                                                        const double *val, const double *R, const double *X,
                                                        double *T) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < (int64_t)n * m;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / m), c = (int)(o % m);
    double q = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) q += val[e] * X[(int64_t)ci[e] * m + c];
    T[o] = R[o] - q;
  }
}

// Rc = P^T T (coarse row I gathers its P^T entries)
__global__ void __launch_bounds__(kBlock) k_cols_restrict(int nc, int m, const int32_t *ptp, const int32_t *pti,
                                                           const double *ptval, const double *T, double *Rc) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < (int64_t)nc * m;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(o / m), c = (int)(o % m);
    double q = 0;
    for (int k = ptp[I]; k < ptp[I + 1]; ++k) q += ptval[k] * T[(int64_t)pti[k] * m + c];
    Rc[o] = q;
  }
}

// Y = X + P Xc (Y may be X)
__global__ void __launch_bounds__(kBlock) k_cols_prolong(int n, int m, const int32_t *prp, const int32_t *pci,
                                                          const double *pval, const double *Xc, const double *X,
                                                          double *Y) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < (int64_t)n * m;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / m), c = (int)(o % m);
    double q = 0;
    for (int e = prp[i]; e < prp[i + 1]; ++e) q += pval[e] * Xc[(int64_t)pci[e] * m + c];
    Y[o] = X[o] + q;
  }
}

// X = Ainv R (dense n x n times n x m)
__global__ void __launch_bounds__(kBlock) k_cols_dense(int n, int m, const double *Ainv, const double *R,
                                                        double *X) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < (int64_t)n * m;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(o / m), c = (int)(o % m);
    double q = 0;
    for (int j = 0; j < n; ++j) q += Ainv[(int64_t)i * n + j] * R[(int64_t)j * m + c];
    X[o] = q;
  }
}

}  // namespace

int amg_group(double avg);

// Column-block V-cycle on level l: X_l = V_l(R_l) for the m columns of cr[l]
// (result in cx[l]); the steps of the vector V-cycle.
static void cols_vcycle(const AmgDev &A, int l, int m, int nu, hipStream_t s) {
  const AmgDevLevel &L = A.lev[l];
  const int n = L.n;
  const dim3 b(kBlock), g(grid_for((int64_t)n * m));
  double *R = A.cr[l], *X = A.cx[l], *T = A.ct[l];
  auto sweep = [&](const double *xin, double *xout, int half) {
    hipLaunchKernelGGL(k_cols_sweep, g, b, 0, s, n, m, L.rp, L.ci, (const double *)L.val, (const double *)L.dinv,
                       (const double *)L.lam, (const double *)R, xin, xout, half);
  };
  if (l == A.nlev - 1) {
    if (A.ainv) {
      hipLaunchKernelGGL(k_cols_dense, g, b, 0, s, n, m, (const double *)A.ainv, (const double *)R, X);
      return;
    }
    constexpr int rest = kAmgCoarseSweeps - 2;
    double *cur = (rest % 2 == 1) ? T : X;
    sweep(nullptr, cur, 0);
    for (int it = 0; it < rest; ++it) {
      double *nxt = (cur == X) ? T : X;
      sweep(cur, nxt, 0);
      cur = nxt;
    }
    return;
  }
  const AmgDevLevel &N = A.lev[l + 1];
  sweep(nullptr, X, nu == 1);  // pre-smoothing from zero
  hipLaunchKernelGGL(k_cols_resid, g, b, 0, s, n, m, L.rp, L.ci, (const double *)L.val, (const double *)R,
                     (const double *)X, T);
  hipLaunchKernelGGL(k_cols_restrict, dim3(grid_for((int64_t)N.n * m)), b, 0, s, N.n, m, L.ptp, L.pti,
                     (const double *)L.ptval, (const double *)T, A.cr[l + 1]);
  cols_vcycle(A, l + 1, m, nu, s);
  // prolongation, then nu post-sweeps alternating between T and X, ending in X
  double *cur = (nu % 2 == 1) ? T : X;
  hipLaunchKernelGGL(k_cols_prolong, g, b, 0, s, n, m, L.prp, L.pci, (const double *)L.pval,
                     (const double *)A.cx[l + 1], (const double *)X, cur);
  for (int it = 0; it < nu; ++it) {
    double *nxt = (cur == X) ? T : X;
    sweep(cur, nxt, 0);
    cur = nxt;
  }
}

void amg_numeric_setup(const AmgDev &A, int cond, int d, int bs, int64_t nnzb0, const double *bsr0, int nu,
                       int *err, hipStream_t s) {
  hipLaunchKernelGGL(k_amg_extract0, dim3(grid_for(nnzb0)), dim3(kBlock), 0, s, nnzb0, bs, d, cond, bsr0,
                     A.lev[0].val);
  for (int l = 0; l < A.nlev; ++l) {
    const AmgDevLevel &L = A.lev[l];
    if (l == A.nlev - 1 && A.ainv) {
      const size_t lds = ((size_t)L.n * L.n + 2 * L.n) * sizeof(double);
      static bool attr = false;
      if (!attr) {
        if (hipFuncSetAttribute((const void *)k_amg_coarsest_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(kMaxLdsBytes - 1024)) != hipSuccess)
          fail(HHO_E_DEVICE, "AMG coarsest: cannot reserve LDS");
        attr = true;
      }
      if (lds <= kMaxLdsBytes - 1024)
        hipLaunchKernelGGL(k_amg_coarsest_lds, dim3(1), dim3(1024), lds, s, L.n, L.rp, L.ci,
                           (const double *)L.val, A.ainv, err);
      else
        hipLaunchKernelGGL(k_amg_coarsest, dim3(1), dim3(kBlock), 0, s, L.n, L.rp, L.ci, L.val, A.dense_scratch,
                           A.ainv, err);
      break;
    }
    const int GA = amg_group((double)L.nnz / L.n);
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(grid_for((int64_t)L.n * GA), 256));
    hipLaunchKernelGGL(k_amg_diag, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.diag, (const double *)L.val,
                       L.dinv, L.tmp);
    // lambda ~ rho(D^{-1} A) by power iteration (vectors ping-pong between tmp
    // and res, partial sums between the two halves of the partial buffer)
    for (int k = 0; k < kAmgPowerSteps; ++k) {
      const double *vin = (k % 2 == 0) ? L.tmp : L.res;
      double *vout = (k % 2 == 0) ? L.res : L.tmp;
      const double *pin = A.partial + ((k + 1) % 2) * 256;
      double *pout = A.partial + (k % 2) * 256;
#define HHO_PW(GG)                                                                                             \
  hipLaunchKernelGGL((k_amg_power<GG>), dim3(nb), dim3(kBlock), 0, s, L.n, L.rp, L.ci, (const double *)L.val,   \
                     (const double *)L.dinv, vin, pin, k ? nb : 0, vout, pout)
      switch (GA) {
        case 64: HHO_PW(64); break;
        case 16: HHO_PW(16); break;
        case 4: HHO_PW(4); break;
        default: HHO_PW(1); break;
      }
#undef HHO_PW
    }
    hipLaunchKernelGGL(k_amg_power_finish, dim3(1), dim3(kBlock), 0, s, nb,
                       (const double *)(A.partial + ((kAmgPowerSteps - 1) % 2) * 256), L.lam, kAmgLambdaSafety);
    if (l == A.nlev - 1) break;  // large coarsest level: Jacobi sweeps only
    if (L.np1 > 0) {  // two smoothing steps
      hipLaunchKernelGGL(k_amg_p, dim3(grid_for(L.np1)), dim3(kBlock), 0, s, (int64_t)L.np1, L.p1row, L.pgp, L.pgi,
                         L.pself, L.val, L.dinv, L.lam, L.pval1);
      hipLaunchKernelGGL(k_amg_pairs, dim3(grid_for(L.npe)), dim3(kBlock), 0, s, L.npe, L.qpp, L.qpa, L.qpb,
                         (const double *)L.val, (const double *)L.pval1, L.qval);
      hipLaunchKernelGGL(k_amg_p2, dim3(grid_for(L.npe)), dim3(kBlock), 0, s, L.npe, L.p2src, L.prow,
                         (const double *)L.pval1, (const double *)L.qval, (const double *)L.dinv,
                         (const double *)L.lam, L.pval);
    } else {
      hipLaunchKernelGGL(k_amg_p, dim3(grid_for(L.npe)), dim3(kBlock), 0, s, L.npe, L.prow, L.pgp, L.pgi, L.pself,
                         L.val, L.dinv, L.lam, L.pval);
    }
    hipLaunchKernelGGL(k_amg_pairs, dim3(grid_for(L.nbe)), dim3(kBlock), 0, s, L.nbe, L.bpp, L.bpa, L.bpb,
                       (const double *)L.val, (const double *)L.pval, L.bval);
    const AmgDevLevel &N = A.lev[l + 1];
    hipLaunchKernelGGL(k_amg_pairs, dim3(grid_for(N.nnz)), dim3(kBlock), 0, s, N.nnz, L.cpp, L.cpa, L.cpb,
                       (const double *)L.pval, (const double *)L.bval, N.val);
    hipLaunchKernelGGL(k_amg_gather, dim3(grid_for(L.npe)), dim3(kBlock), 0, s, L.npe, L.pte,
                       (const double *)L.pval, L.ptval);
    hipLaunchKernelGGL(k_amg_gather, dim3(grid_for(L.nbe)), dim3(kBlock), 0, s, L.nbe, L.bte,
                       (const double *)L.bval, L.btval);
  }
  if (A.expl >= 0) {  // M = V_expl(I)
    const int m = A.lev[A.expl].n;
    hipLaunchKernelGGL(k_cols_identity, dim3(grid_for((int64_t)m * m)), dim3(kBlock), 0, s, (int64_t)m,
                       A.cr[A.expl]);
    cols_vcycle(A, A.expl, m, nu, s);  // M is cx[expl]
  }
}

void bp_setup(const DTopo &tp, int cond, const int32_t *fdiag, const double *bsr, const double *cpl, double *Sd,
              hipStream_t s) {
  hipLaunchKernelGGL(k_bp_setup, dim3(grid_for(tp.nc)), dim3(kBlock), 0, s, tp, cond, fdiag, bsr, cpl, Sd);
}

// V-cycle on level l: x = AMG_l(r); x, r are [n_l][d].  nu damped-Jacobi sweeps
// before and after the coarse correction (nu = 1 or 2).
static void rows(int G, int n, int d, const AmgDevLevel &L, const double *r, const double *xin, double *xout,
                 hipStream_t s, const int *skip) {
  const dim3 b(kBlock), g(grid_for((int64_t)n * G));
  const double *val = L.val, *dinv = L.dinv, *lam = L.lam;
  switch (G) {
    case 64: HHO_LAUNCH((k_amg_rows<64>), g, b, 0, s, n, d, L.rp, L.ci, val, dinv, lam, r, xin, xout, skip); break;
    case 16: HHO_LAUNCH((k_amg_rows<16>), g, b, 0, s, n, d, L.rp, L.ci, val, dinv, lam, r, xin, xout, skip); break;
    case 4: HHO_LAUNCH((k_amg_rows<4>), g, b, 0, s, n, d, L.rp, L.ci, val, dinv, lam, r, xin, xout, skip); break;
    default: HHO_LAUNCH((k_amg_rows<1>), g, b, 0, s, n, d, L.rp, L.ci, val, dinv, lam, r, xin, xout, skip); break;
  }
}

static void prolong_sweep(int G, const AmgDevLevel &L, int d, const double *xc, const double *r, const double *xin,
                          double *xout, hipStream_t s, const int *skip) {
  const dim3 b(kBlock), g(grid_for((int64_t)L.n * G));
#define HHO_PS(GG)                                                                                             \
  HHO_LAUNCH((k_amg_prolong_sweep<GG>), g, b, 0, s, L.n, d, L.rp, L.ci, (const double *)L.val,           \
                     (const double *)L.dinv, (const double *)L.lam, L.prp, L.pci, (const double *)L.pval, L.brp, \
                     L.bci, (const double *)L.bval, xc, r, xin, xout, skip)
  switch (G) {
    case 64: HHO_PS(64); break;
    case 16: HHO_PS(16); break;
    case 4: HHO_PS(4); break;
    default: HHO_PS(1); break;
  }
#undef HHO_PS
}

// lanes per row for a given average row length
int amg_group(double avg) { return avg >= 48 ? 64 : avg >= 12 ? 16 : avg >= 3 ? 4 : 1; }

// V-cycle on level l: x = AMG_l(r); x, r are [n_l][d].  nu damped-Jacobi sweeps
// before and after the coarse correction (nu = 1 or 2).
static void vcycle(const AmgDev &A, int l, int d, int nu, const double *r, double *x, hipStream_t s,
                   const int *skip) {
  const AmgDevLevel &L = A.lev[l];
  if (l == A.expl) {  // this level and all coarser ones: the explicit operator
    HHO_PROBED(A.probe, HHO_PROBE_AMG_DENSE, l, s,
               HHO_LAUNCH(k_amg_dense, dim3(L.n), dim3(kBlock), 0, s, L.n, d, (const double *)A.mexpl, r, x, skip));
    return;
  }
  if (l == A.nlev - 1) {
    if (A.ainv) {
      HHO_PROBED(A.probe, HHO_PROBE_AMG_DENSE, l, s,
                 HHO_LAUNCH(k_amg_dense, dim3(L.n), dim3(kBlock), 0, s, L.n, d, (const double *)A.ainv, r, x, skip));
      return;
    }
    // kAmgCoarseSweeps damped-Jacobi sweeps from zero (the first launch takes two)
    const int GA = amg_group((double)L.nnz / L.n);
    constexpr int rest = kAmgCoarseSweeps - 2;
    double *cur = (rest % 2 == 1) ? L.tmp : x;
    HHO_PROBED(A.probe, HHO_PROBE_AMG_SWEEP, l, s, rows(GA, L.n, d, L, r, nullptr, cur, s, skip));
    for (int it = 0; it < rest; ++it) {
      double *nxt = (cur == x) ? L.tmp : x;
      HHO_PROBED(A.probe, HHO_PROBE_AMG_SWEEP, l, s, rows(GA, L.n, d, L, r, cur, nxt, s, skip));
      cur = nxt;
    }
    return;
  }
  const AmgDevLevel &N = A.lev[l + 1];
  const int GA = amg_group((double)L.nnz / L.n), GS = amg_group((double)std::max(L.nnz, L.nbe) / L.n);
  // pre-smoothing from zero: for nu = 2 one launch takes both sweeps; for nu = 1
  // the single sweep x = w D^{-1} r is formed where it is used
  const double *xpre = nullptr;
  if (nu == 2) {
    HHO_PROBED(A.probe, HHO_PROBE_AMG_SWEEP, l, s, rows(GA, L.n, d, L, r, nullptr, x, s, skip));
    xpre = x;
  }
  HHO_PROBED(A.probe, HHO_PROBE_AMG_RESTRICT, l, s,
             HHO_LAUNCH(k_amg_restrict, dim3(grid_for((int64_t)N.n * kWave)), dim3(kBlock), 0, s, N.n, d,
                                L.ptp, L.pti, (const double *)L.ptval, L.btp, L.bti, (const double *)L.btval,
                                (const double *)L.dinv, (const double *)L.lam, r, xpre, N.r, skip));
  vcycle(A, l + 1, d, nu, N.r, N.x, s, skip);
  // prolongation with the first post-sweep (nu = 2: into tmp, then the second sweep into x)
  HHO_PROBED(A.probe, HHO_PROBE_AMG_PROLONG, l, s, prolong_sweep(GS, L, d, N.x, r, xpre, nu == 2 ? L.tmp : x, s, skip));
  if (nu == 2) HHO_PROBED(A.probe, HHO_PROBE_AMG_SWEEP, l, s, rows(GA, L.n, d, L, r, L.tmp, x, s, skip));
}

void bp_apply(const DTopo &tp, const AmgDev &A, int64_t nface, const double *cpl, const double *Sd, const double *v,
              double *z, int nu, hipStream_t s, const int *skip) {
  const int d = tp.d;
  hipLaunchKernelGGL(k_bp_rhs, dim3(grid_for(nface + tp.nc)), dim3(kBlock), 0, s, tp, nface, cpl, Sd, v,
                     A.lev[0].r, z, skip);
  vcycle(A, 0, d, nu, A.lev[0].r, z, s, skip);
}

}  // namespace hho
