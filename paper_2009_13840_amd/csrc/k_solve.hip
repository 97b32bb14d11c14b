// Solve-phase kernels: face-block operator application, cell-patch Schwarz
// preconditioner, matrix-free intergrid transfers (Section 3.1: truncation and
// zero-padded injection), the smoother's minimal-residual step, and the
// reductions of the Arnoldi process.  Templated on the vector/operator type
// (FP64, or FP32 for the mixed-precision V-cycle); reductions accumulate in FP64.
#include <algorithm>
#include <cmath>

#include "dev_common.h"
#include "device.h"
#include "probe.h"
#include "internal.h"

namespace hho {
namespace {

inline int grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

template <typename T, bool SPLIT>
__device__ inline T xface(const T *x, const T *xs1, int64_t i) {
  if (SPLIT) return x[i] + xs1[i];
  return x[i];
}

// y = S x  (MODE 0)   or   y = b - S x  (MODE 1).  One thread per output entry:
// face rows first (f, c, r), then cell rows (T, q).
template <typename T, typename Sto, typename StoP, bool SPLIT, int MODE>
__global__ void __launch_bounds__(kBlock) k_spmv(DTopo tp, DLevel<T, Sto, StoP> L, const T *__restrict__ x,
                                                  const T *__restrict__ xs1, T *__restrict__ xsum,
                                                  const T *__restrict__ b, T *__restrict__ y) {
  const int d = tp.d, p = L.p, t = L.t;
  const int dp = d * p;
  const int64_t total = L.N;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total; o += (int64_t)gridDim.x * blockDim.x) {
    T acc = 0;
    if (o < L.nface) {
      const int f = (int)(o / dp);
      const int cr = (int)(o % dp);
      const int rb = tp.rowptr[f], re = tp.rowptr[f + 1];
      if (L.cond == 1) {
        const int c = cr / p, r = cr % p;
        for (int b = rb; b < re; ++b) {
          const Sto *blk = L.bsr + (int64_t)b * p * p + r * p;
          const int64_t xo = ((int64_t)tp.col[b] * d + c) * p;
          for (int k = 0; k < p; ++k) acc += blk[k] * xface<T, SPLIT>(x, xs1, xo + k);
        }
        for (int s = 0; s < 2; ++s) {
          const int Tc = tp.fcell[2 * f + s];
          if (Tc < 0) continue;
          const int64_t e = (int64_t)tp.cptr[Tc] + tp.floc[2 * f + s];
          const Sto *cp = L.cpl + ((e * d + c) * p + r) * t;
          const T *xp = x + L.nface + (int64_t)Tc * t;
          for (int q = 0; q < t; ++q) acc += cp[q] * xp[q];
        }
      } else {
        for (int b = rb; b < re; ++b) {
          const Sto *blk = L.bsr + (int64_t)b * dp * dp + (int64_t)cr * dp;
          const int64_t xo = (int64_t)tp.col[b] * dp;
          for (int k = 0; k < dp; ++k) acc += blk[k] * xface<T, SPLIT>(x, xs1, xo + k);
        }
        for (int s = 0; s < 2; ++s) {
          const int Tc = tp.fcell[2 * f + s];
          if (Tc < 0) continue;
          const int64_t e = (int64_t)tp.cptr[Tc] + tp.floc[2 * f + s];
          acc += L.cpl[e * dp + cr] * x[L.nface + Tc];
        }
      }
      if (SPLIT && xsum) xsum[o] = xface<T, SPLIT>(x, xs1, o);
    } else {
      const int64_t oc = o - L.nface;
      const int Tc = (int)(oc / t), q = (int)(oc % t);
      const int eb = tp.cptr[Tc], ee = tp.cptr[Tc + 1];
      if (L.cond == 1) {
        for (int e = eb; e < ee; ++e) {
          const int64_t xo = (int64_t)tp.cface[e] * dp;
          const Sto *cp = L.cpl + (int64_t)e * dp * t + q;
          for (int k = 0; k < dp; ++k) acc += cp[(int64_t)k * t] * xface<T, SPLIT>(x, xs1, xo + k);
        }
        const Sto *sp = L.spp + ((int64_t)Tc * t + q) * t;
        const T *xp = x + L.nface + (int64_t)Tc * t;
        for (int q2 = 0; q2 < t; ++q2) acc += sp[q2] * xp[q2];
      } else {
        for (int e = eb; e < ee; ++e) {
          const int64_t xo = (int64_t)tp.cface[e] * dp;
          const Sto *cp = L.cpl + (int64_t)e * dp;
          for (int k = 0; k < dp; ++k) acc += cp[k] * xface<T, SPLIT>(x, xs1, xo + k);
        }
      }
      if (SPLIT && xsum) xsum[o] = x[o];
    }
    y[o] = (MODE == 1) ? (T)(b[o] - acc) : acc;
  }
}

// y = (S (x) I_d) x for a symmetric m x m matrix S (m <= 64 SM) stored as its
// lower triangle packed by rows (entry (i, j), i >= j, at i (i + 1) / 2 + j).
// The vectors are in LDS in the patch order [(face, component, mode)] with p
// modes per face and DC components (DC = 1, p = m: a plain product).  One
// wavefront: every row j of the triangle is read once, coalesced; its strictly
// lower entries add S_ji x_j to y_i (S_ij = S_ji, lane-local), and the whole row
// gives y_j's dot product.  R rows are loaded together (R * SM loads in flight)
// and their R * DC dot products are reduced across the wave together.
template <typename T, typename Sto, int SM, int DC>
__device__ void sym_packed_apply(const Sto *__restrict__ S, int m, int p, const T *x, T *y, T *ydot) {
  constexpr int DCP = DC == 1 ? 1 : DC == 2 ? 2 : 4;  // components padded to a power of two
  constexpr int R = (SM >= 3 ? 4 : 8) / DCP > 0 ? (SM >= 3 ? 4 : 8) / DCP : 1;  // rows per group
  constexpr int NV = R * DCP;                                                   // sums reduced together
  constexpr int shift = 6 - log2i<NV>();
  const int lane = threadIdx.x;
  T acc[SM][DC], xi[SM][DC];
#pragma unroll
  for (int s = 0; s < SM; ++s) {
    const int i = lane + s * kWave;
    const int ib = (i < m) ? ((i / p) * DC) * p + i % p : 0;
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      acc[s][c] = 0;
      xi[s][c] = (i < m) ? x[ib + c * p] : (T)0;
    }
  }
  int jf = 0, jr = 0;  // j0 = jf p + jr
  for (int j0 = 0; j0 < m; j0 += R) {
    T v[R][SM];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = j0 + r;
      const Sto *row = S + (int64_t)j * (j + 1) / 2;
#pragma unroll
      for (int s = 0; s < SM; ++s) {
        const int i = lane + s * kWave;
        v[r][s] = (j < m && i <= j) ? (T)row[i] : (T)0;
      }
    }
    T dot[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) dot[q] = 0;
    int f = jf, rr = jr;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = j0 + r;
      if (j < m) {
        const int jb = (f * DC) * p + rr;
#pragma unroll
        for (int c = 0; c < DC; ++c) {
          const T xj = x[jb + c * p];
          T dsum = 0;
#pragma unroll
          for (int s = 0; s < SM; ++s) {
            const int i = lane + s * kWave;
            dsum += v[r][s] * xi[s][c];
            acc[s][c] += ((i < j) ? v[r][s] : (T)0) * xj;
          }
          dot[r * DCP + c] = dsum;
        }
      }
      if (++rr == p) {
        rr = 0;
        ++f;
      }
    }
    jf = f;
    jr = rr;
    wave_multi_sum<NV>(dot);
    if ((lane & ((1 << shift) - 1)) == 0) {
      const int q = lane >> shift, r = q / DCP, c = q % DCP;
      if (c < DC && j0 + r < m) ydot[c * m + j0 + r] = dot[0];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SM; ++s) {
    const int i = lane + s * kWave;
    if (i < m) {
      const int ib = ((i / p) * DC) * p + i % p;
#pragma unroll
      for (int c = 0; c < DC; ++c) y[ib + c * p] = acc[s][c] + ydot[c * m + i];
    }
  }
  __syncthreads();
}

// The same product for patches of at most 64 rows: one thread per row i walks
// its whole row through the packed index (the triangle stays in the L1/L2 caches
// after its first touch) and forms that row's DC outputs, so that each entry of
// the triangle is loaded by one lane; no cross-lane reduction.
template <typename T, typename Sto, int DC>
__device__ void sym_row_apply(const Sto *__restrict__ S, int m, int p, const T *x, T *y) {
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const int fi = i / p, rr = i % p;
    T acc[DC];
#pragma unroll
    for (int c = 0; c < DC; ++c) acc[c] = 0;
    int jf = 0, jr = 0;
#pragma unroll 8
    for (int j = 0; j < m; ++j) {
      const int lo = j < i ? j : i, hi = j < i ? i : j;
      const T sij = (T)S[hi * (hi + 1) / 2 + lo];
#pragma unroll
      for (int c = 0; c < DC; ++c) acc[c] += sij * x[(jf * DC + c) * p + jr];
      if (++jr == p) {
        jr = 0;
        ++jf;
      }
    }
#pragma unroll
    for (int c = 0; c < DC; ++c) y[(fi * DC + c) * p + rr] = acc[c];
  }
  __syncthreads();
}

// Cell-patch Schwarz preconditioner; one 64-thread block per cell.  The
// corrections of the face unknowns are weighted by 1/card(T_F) and written to the
// slot of the face's side (slot 0: first cell of the face -> z, slot 1 -> zs1), so
// that z_F = slot 0 + slot 1 with no write conflict.
// SM, DC: as sym_packed_apply for the level's largest patch (DC = d for v-cond, 1 for v&p).
template <typename T, typename Sto, typename StoP, int SM, int DC>
__global__ void __launch_bounds__(kWave) k_precond(DTopo tp, DLevel<T, Sto, StoP> L, const T *__restrict__ r,
                                                   const double *__restrict__ scale, T *__restrict__ v,
                                                   T *__restrict__ z, T *__restrict__ zs1) {
  extern __shared__ unsigned char smem[];
  T *sh = (T *)smem;
  const int Tc = blockIdx.x;
  const int d = tp.d, p = L.p, t = L.t, dp = d * p;
  const int eb = tp.cptr[Tc], nfc = tp.cptr[Tc + 1] - eb;
  const int m = nfc * p, n = nfc * dp;
  const T sc = scale ? (T)scale[0] : (T)1;
  T *ru = sh;                  // [n] patch residual (face part)
  T *u1 = ru + n;              // [n]
  T *wv = u1 + n;              // [max(n, t)]
  T *yp = wv + (n > t ? n : t);  // [t + 1]
  T *rpr = yp + t + 1;         // [t]
  T *ydot = rpr + t;           // [n]
  T *red = ydot + n;           // [64] partial sums
  int *fl = (int *)(red + kWave);  // [2 n] face of each patch row, and its sides (2: first cell is Tc, 1: interior)
  const StoP *Si = L.sinv + tp.pairoff[Tc] * (int64_t)((L.cond == 1) ? p * p : dp * dp);  // packed lower triangle
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int fi = i / dp, k = i % dp;
    const int f = tp.cface[eb + fi];
    const T val = sc * r[(int64_t)f * dp + k];
    const int c0 = tp.fcell[2 * f], c1 = tp.fcell[2 * f + 1];  // read with r, kept for the write-back
    ru[i] = val;
    fl[2 * i] = f;
    fl[2 * i + 1] = (c0 == Tc ? 2 : 0) | (c1 >= 0 ? 1 : 0);
    if (v && c0 == Tc) v[(int64_t)f * dp + k] = val;
  }
  for (int q = threadIdx.x; q < t; q += blockDim.x) {
    const T val = sc * r[L.nface + (int64_t)Tc * t + q];
    rpr[q] = val;
    if (v) v[L.nface + (int64_t)Tc * t + q] = val;
  }
  __syncthreads();
  if (L.cond == 1) {
    const Sto *C = L.cpl + (int64_t)eb * dp * t;      // [n][t]
    // u1 = (s^{-1} (x) I) r_u
    if constexpr (SM == 1) sym_row_apply<T, StoP, DC>(Si, m, p, ru, u1);
    else sym_packed_apply<T, StoP, SM, DC>(Si, m, p, ru, u1, ydot);
    // y_p = X^{-1} (r_p - C^T u1); C^T u1 by lanes (part, q), parts = 64 / t taking
    // every parts-th row (coalesced rows of C), partials combined in order
    if (t <= kWave) {
      const int parts = kWave / t, q = threadIdx.x % t, part = threadIdx.x / t;
      T acc = 0;
      if (part < parts)
#pragma unroll 8
        for (int i = part; i < n; i += parts) acc += C[(int64_t)i * t + q] * u1[i];
      red[threadIdx.x] = acc;
      __syncthreads();
      if (threadIdx.x < t) {
        T s = rpr[threadIdx.x];
        for (int pp = 0; pp < parts; ++pp) s -= red[pp * t + threadIdx.x];
        wv[threadIdx.x] = s;
      }
    } else {
      for (int q = threadIdx.x; q < t; q += blockDim.x) {
        T acc = rpr[q];
        for (int i = 0; i < n; ++i) acc -= C[(int64_t)i * t + q] * u1[i];
        wv[q] = acc;
      }
    }
    __syncthreads();
    const StoP *Xi = L.xinv + (int64_t)Tc * t * t;
    for (int q = threadIdx.x; q < t; q += blockDim.x) {
      T acc = 0;
      for (int q2 = 0; q2 < t; ++q2) acc += Xi[q * t + q2] * wv[q2];
      yp[q] = acc;
    }
    __syncthreads();
    // w = r_u - C y_p ; y_u = (s^{-1} (x) I) w
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      T acc = ru[i];
#pragma unroll 8
      for (int q = 0; q < t; ++q) acc -= C[(int64_t)i * t + q] * yp[q];
      wv[i] = acc;
    }
    __syncthreads();
    if constexpr (SM == 1) sym_row_apply<T, StoP, DC>(Si, m, p, wv, u1);
    else sym_packed_apply<T, StoP, SM, DC>(Si, m, p, wv, u1, ydot);
  } else {
    const StoP *g = L.xinv + (int64_t)eb * dp;
    if constexpr (SM == 1) sym_row_apply<T, StoP, DC>(Si, n, n, ru, u1);
    else sym_packed_apply<T, StoP, SM, DC>(Si, n, n, ru, u1, ydot);
    T part = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) part += g[i] * ru[i];
    // wave reduction (blockDim == 64)
    double pd = wave_sum((double)part);
    if (threadIdx.x == 0) yp[0] = (T)((pd - (double)rpr[0]) * (double)(T)L.sig[Tc]);
    __syncthreads();
    const T ypv = yp[0];
    for (int i = threadIdx.x; i < n; i += blockDim.x) u1[i] -= g[i] * ypv;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int k = i % dp;
    const int f = fl[2 * i];
    const bool first = fl[2 * i + 1] & 2;
    const bool interior = fl[2 * i + 1] & 1;
    const T val = interior ? (T)0.5 * u1[i] : u1[i];
    if (first) {
      z[(int64_t)f * dp + k] = val;
      if (!interior) zs1[(int64_t)f * dp + k] = (T)0;  // no second side on the boundary
    } else {
      zs1[(int64_t)f * dp + k] = val;
    }
  }
  for (int q = threadIdx.x; q < t; q += blockDim.x) z[L.nface + (int64_t)Tc * t + q] = yp[q];
}

template <typename T>
__global__ void k_combine(int64_t nface, const T *zs1, T *z) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nface; i += (int64_t)gridDim.x * blockDim.x)
    z[i] += zs1[i];
}

// restriction (truncation to the leading modes) and prolongation (zero-padded add)
template <typename Tc, typename Tf, bool ADD>
__global__ void k_transfer(int d, int nf, int nc, int pf, int tf, int pc, int tc, const Tf *xf, Tc *xc, Tf *xfo,
                           const Tc *xci) {
  const int64_t nfc = (int64_t)nf * d * pc;
  const int64_t total = nfc + (int64_t)nc * tc;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t j;
    if (i < nfc) {
      const int64_t fcmp = i / pc;
      j = fcmp * pf + i % pc;
    } else {
      const int64_t k = i - nfc;
      j = (int64_t)nf * d * pf + (k / tc) * tf + k % tc;
    }
    if (ADD)
      xfo[j] += (Tf)xci[i];
    else
      xc[i] = (Tc)xf[j];
  }
}

// ---- smoother: minimal residual over span{z1, z2} (the GMRES(2) iterate)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mr2_dots(int64_t n, int m, const T *w1, const T *w2, const T *r,
                                                      double *partial) {
  __shared__ double red[16];
  double a11 = 0, a12 = 0, a22 = 0, g1 = 0, g2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x1 = w1[i], rr = r[i];
    a11 += x1 * x1;
    g1 += x1 * rr;
    if (m == 2) {
      const double x2 = w2[i];
      a12 += x1 * x2;
      a22 += x2 * x2;
      g2 += x2 * rr;
    }
  }
  double v[5] = {a11, a12, a22, g1, g2};
  for (int k = 0; k < 5; ++k) {
    double s = block_sum(v[k], red);
    if (threadIdx.x == 0) partial[k * gridDim.x + blockIdx.x] = s;
  }
}

// y = G^{-1} g from the partial sums of k_mr2_dots (one block)
__global__ void __launch_bounds__(kBlock) k_mr2_finish(int G, int m, const double *partial, double *y) {
  __shared__ double S[5];
  reduce_partials(partial, G, 5, S);
  if (threadIdx.x == 0) mr2_solve(S, m, y);
}

template <typename T>
__global__ void k_mr2_update(int64_t n, int m, const double *y, const T *z1, const T *z2, const T *w1, const T *w2,
                             T *x, T *r) {
  const T y1 = (T)y[0], y2 = (T)y[1];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (m == 2) {
      x[i] += y1 * z1[i] + y2 * z2[i];
      r[i] -= y1 * w1[i] + y2 * w2[i];
    } else {
      x[i] += y1 * z1[i];
      r[i] -= y1 * w1[i];
    }
  }
}

// |r|^2 partial sums
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sumsq(int64_t n, const T *r, double *partial) {
  __shared__ double red[16];
  double acc = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double v = r[k];
    acc += v * v;
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// |r| -> beta (and bnorm if which == 1), g = beta e1, reset the cycle (one block).
__global__ void __launch_bounds__(kBlock) k_norm_finish(int G, const double *partial, GmresState *st, int which) {
  __shared__ double nsum[1];
  reduce_partials(partial, G, 1, nsum);
  if (threadIdx.x == 0) {
    const double nn = nsum[0];
    const double beta = sqrt(nn);
    st->beta = beta;
    if (which == 1) {
      st->bnorm = beta;
      st->its = 0;
    }
    for (int i = 0; i <= kMaxRestartH; ++i) st->g[i] = 0;
    st->g[0] = beta;
    st->res = beta;
    st->j = 0;
    st->inv_hnext = (beta > 0) ? 1.0 / beta : 0.0;
    st->nan = !isfinite(nn);
    st->done = (!(beta > 0) || st->nan || beta <= st->rtol * st->bnorm) ? 1 : 0;
  }
}

template <typename T>
__global__ void k_scale(int64_t n, const T *x, const double *scale, T *y) {
  const T s = (T)scale[0];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = s * x[k];
}

// y = H^{-1} g over the st->j columns of the current cycle (single thread)
__global__ void k_gmres_solve_ls(GmresState *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int R = kMaxRestartH;
  const int jn = st->j;
  for (int i = jn - 1; i >= 0; --i) {
    double v = st->g[i];
    for (int k = i + 1; k < jn; ++k) v -= st->H[i * R + k] * st->y[k];
    const double hii = st->H[i * R + i];
    st->y[i] = (hii != 0) ? v / hii : 0.0;
  }
}

template <typename T>
__global__ void k_gmres_combine(int64_t n, const T *Z, int64_t ldz, const GmresState *st, T *x) {
  const int jn = st->j;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double v = x[k];
    for (int i = 0; i < jn; ++i) v += st->y[i] * (double)Z[i * ldz + k];
    x[k] = (T)v;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot(int64_t n, const T *a, const T *b, double *partial) {
  __shared__ double red[16];
  double acc = 0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    acc += (double)a[k] * (double)b[k];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_sum_finish(int G, const double *partial, double *out) {
  __shared__ double vs[1];
  reduce_partials(partial, G, 1, vs);
  if (threadIdx.x == 0) out[0] = vs[0];
}

// y += sign * (alpha[0] / alpha[1]) * x  (alpha[1] = 1 when not a ratio)
template <typename T>
__global__ void k_axpy_ratio(int64_t n, const double *alpha, double sign, const T *x, T *y) {
  const double a = sign * alpha[0] / alpha[1];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = (T)((double)y[k] + a * (double)x[k]);
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T *x) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    x[k] = v;
}
template <typename T>
__global__ void k_copy(int64_t n, const T *x, T *y) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = x[k];
}

}  // namespace

// ------------------------------------------------------------ wrappers
int reduce_blocks(int64_t n) {
  int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 256));
}

template <typename T, typename Sto, typename StoP>
void launch_spmv(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *x, const T *xs1, T *xsum, T *y, hipStream_t s) {
  if (launch_spmv_fixed<T, Sto, StoP>(tp, L, x, xs1, xsum, nullptr, y, s)) return;
  if (xs1)
    HHO_LAUNCH((k_spmv<T, Sto, StoP, true, 0>), dim3(grid_for(L.N)), dim3(kBlock), 0, s, tp, L, x, xs1, xsum,
                       (const T *)nullptr, y);
  else
    HHO_LAUNCH((k_spmv<T, Sto, StoP, false, 0>), dim3(grid_for(L.N)), dim3(kBlock), 0, s, tp, L, x, xs1, xsum,
                       (const T *)nullptr, y);
}
template <typename T, typename Sto, typename StoP>
void launch_residual(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *b, const T *x, T *r, hipStream_t s) {
  if (launch_spmv_fixed<T, Sto, StoP>(tp, L, x, nullptr, nullptr, b, r, s)) return;
  hipLaunchKernelGGL((k_spmv<T, Sto, StoP, false, 1>), dim3(grid_for(L.N)), dim3(kBlock), 0, s, tp, L, x, (const T *)nullptr,
                     (T *)nullptr, b, r);
}
size_t precond_lds_bytes(int d, int cond, int p, int t, int max_faces, size_t elem) {
  const int n = max_faces * d * p;
  return (size_t)(3 * n + std::max(n, t) + 2 * t + 2 + kWave) * elem + 2 * n * sizeof(int);
}
template <typename T, typename Sto, typename StoP>
void launch_precond(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *r, const double *scale, T *v, T *z, T *zs1,
                    int max_faces, hipStream_t s) {
  const size_t lds = precond_lds_bytes(tp.d, L.cond, L.p, L.t, max_faces, sizeof(T));
  const int rows = max_faces * ((L.cond == 1) ? L.p : tp.d * L.p);  // rows of the largest packed inverse
  const int sm = (rows + kWave - 1) / kWave, dc = (L.cond == 1) ? tp.d : 1;
  if (sm < 1 || sm > kPatchMaxRows / kWave) fail(HHO_E_INVALID_ARG, "precond: patch too large");
#define HHO_PC(SM, DC)                                                                                         \
  if (sm == SM && dc == DC) {                                                                                  \
    HHO_LAUNCH((k_precond<T, Sto, StoP, SM, DC>), dim3(tp.nc), dim3(kWave), lds, s, tp, L, r, scale, v, z, zs1); \
    return;                                                                                                    \
  }
  HHO_PC(1, 1) HHO_PC(2, 1) HHO_PC(3, 1) HHO_PC(4, 1)
  HHO_PC(1, 2) HHO_PC(2, 2) HHO_PC(3, 2) HHO_PC(4, 2)
  HHO_PC(1, 3) HHO_PC(2, 3) HHO_PC(3, 3) HHO_PC(4, 3)
#undef HHO_PC
  fail(HHO_E_INVALID_ARG, "precond: no kernel for this patch shape");
}
template <typename T>
void launch_combine(int64_t nface, const T *zs1, T *z, hipStream_t s) {
  hipLaunchKernelGGL((k_combine<T>), dim3(grid_for(nface)), dim3(kBlock), 0, s, nface, zs1, z);
}
template <typename Tc, typename Tf>
void launch_restrict(int d, int nf, int nc, int pf, int tf, int pc, int tc, const Tf *xf, Tc *xc, hipStream_t s) {
  const int64_t total = (int64_t)nf * d * pc + (int64_t)nc * tc;
  hipLaunchKernelGGL((k_transfer<Tc, Tf, false>), dim3(grid_for(total)), dim3(kBlock), 0, s, d, nf, nc, pf, tf, pc,
                     tc, xf, xc, (Tf *)nullptr, (const Tc *)nullptr);
}
template <typename Tc, typename Tf>
void launch_prolong_add(int d, int nf, int nc, int pf, int tf, int pc, int tc, const Tc *xc, Tf *xf,
                        hipStream_t s) {
  const int64_t total = (int64_t)nf * d * pc + (int64_t)nc * tc;
  hipLaunchKernelGGL((k_transfer<Tc, Tf, true>), dim3(grid_for(total)), dim3(kBlock), 0, s, d, nf, nc, pf, tf, pc,
                     tc, (const Tf *)nullptr, (Tc *)nullptr, xf, xc);
}
template <typename T>
void launch_mr2_dots(int64_t n, int m, const T *w1, const T *w2, const T *r, double *partial, double *y,
                     hipStream_t s) {
  const int G = reduce_blocks(n);
  hipLaunchKernelGGL((k_mr2_dots<T>), dim3(G), dim3(kBlock), 0, s, n, m, w1, w2, r, partial);
  hipLaunchKernelGGL(k_mr2_finish, dim3(1), dim3(kBlock), 0, s, G, m, (const double *)partial, y);
}
template <typename T>
void launch_mr2_update(int64_t n, int m, const double *y, const T *z1, const T *z2, const T *w1, const T *w2,
                       T *x, T *r, hipStream_t s) {
  hipLaunchKernelGGL((k_mr2_update<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, m, y, z1, z2, w1, w2, x, r);
}
template <typename T>
void launch_norm_init(int64_t n, const T *r, double *partial, GmresState *st, int which, hipStream_t s) {
  const int G = reduce_blocks(n);
  hipLaunchKernelGGL((k_sumsq<T>), dim3(G), dim3(kBlock), 0, s, n, r, partial);
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(kBlock), 0, s, G, (const double *)partial, st, which);
}
template <typename T>
void launch_scale(int64_t n, const T *x, const double *scale, T *y, hipStream_t s) {
  hipLaunchKernelGGL((k_scale<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, scale, y);
}
void launch_gmres_solve_ls(GmresState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_solve_ls, dim3(1), dim3(64), 0, s, st);
}
template <typename T>
void launch_gmres_combine(int64_t n, const T *Z, int64_t ldz, const GmresState *st, T *x, hipStream_t s) {
  hipLaunchKernelGGL((k_gmres_combine<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, Z, ldz, st, x);
}
template <typename T>
void launch_dot(int64_t n, const T *a, const T *b, double *partial, double *out, hipStream_t s) {
  const int G = reduce_blocks(n);
  hipLaunchKernelGGL((k_dot<T>), dim3(G), dim3(kBlock), 0, s, n, a, b, partial);
  hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kBlock), 0, s, G, (const double *)partial, out);
}
void launch_sum_finish(int G, const double *partial, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kBlock), 0, s, G, partial, out);
}
template <typename T>
void launch_axpy_ratio(int64_t n, const double *alpha, double sign, const T *x, T *y, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy_ratio<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, alpha, sign, x, y);
}
template <typename T>
void launch_fill(int64_t n, T v, T *x, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, v, x);
}
template <typename T>
void launch_copy(int64_t n, const T *x, T *y, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, y);
}

#define HHO_INST_OP(T, Sto, StoP)                                                                               \
  template void launch_spmv<T, Sto, StoP>(const DTopo &, const DLevel<T, Sto, StoP> &, const T *, const T *, T *, \
                                          T *, hipStream_t);                                                     \
  template void launch_residual<T, Sto, StoP>(const DTopo &, const DLevel<T, Sto, StoP> &, const T *, const T *,  \
                                              T *, hipStream_t);                                                 \
  template void launch_precond<T, Sto, StoP>(const DTopo &, const DLevel<T, Sto, StoP> &, const T *,             \
                                             const double *, T *, T *, T *, int, hipStream_t);
HHO_INST_OP(double, double, double)
HHO_INST_OP(float, float, float)
HHO_INST_OP(float, bf16, float)
#undef HHO_INST_OP

#define HHO_INST(T)                                                                                              \
  template void launch_combine<T>(int64_t, const T *, T *, hipStream_t);                                        \
  template void launch_mr2_dots<T>(int64_t, int, const T *, const T *, const T *, double *, double *,           \
                                   hipStream_t);                                                               \
  template void launch_mr2_update<T>(int64_t, int, const double *, const T *, const T *, const T *, const T *,   \
                                     T *, T *, hipStream_t);                                                   \
  template void launch_norm_init<T>(int64_t, const T *, double *, GmresState *, int, hipStream_t);              \
  template void launch_scale<T>(int64_t, const T *, const double *, T *, hipStream_t);                          \
  template void launch_gmres_combine<T>(int64_t, const T *, int64_t, const GmresState *, T *, hipStream_t);     \
  template void launch_dot<T>(int64_t, const T *, const T *, double *, double *, hipStream_t);                  \
  template void launch_axpy_ratio<T>(int64_t, const double *, double, const T *, T *, hipStream_t);             \
  template void launch_fill<T>(int64_t, T, T *, hipStream_t);                                                   \
  template void launch_copy<T>(int64_t, const T *, T *, hipStream_t);
HHO_INST(double)
HHO_INST(float)
#undef HHO_INST

template void launch_restrict<double, double>(int, int, int, int, int, int, int, const double *, double *,
                                              hipStream_t);
template void launch_restrict<float, float>(int, int, int, int, int, int, int, const float *, float *, hipStream_t);
template void launch_restrict<double, float>(int, int, int, int, int, int, int, const float *, double *,
                                             hipStream_t);
template void launch_prolong_add<double, double>(int, int, int, int, int, int, int, const double *, double *,
                                                 hipStream_t);
template void launch_prolong_add<float, float>(int, int, int, int, int, int, int, const float *, float *,
                                               hipStream_t);
template void launch_prolong_add<double, float>(int, int, int, int, int, int, int, const double *, float *,
                                                hipStream_t);

}  // namespace hho
