// Setup kernels: static condensation (eqs. ST.1 / ST.2), assembly of the
// face-block operator (Section 4.2, last paragraph), recursive inheritance of
// the coarse levels by sub-block extraction (Section 4.2), factorisation of the
// smoother's cell patches, and the dense coarse inverse.  All FP64.
#include <algorithm>

#include "dev_common.h"
#include "dev_dense.h"
#include "device.h"
#include "internal.h"

namespace hho {
namespace {

// ------------------------------------------------------------ V-cycle copy by a matrix-core product
typedef short v4bf __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

__device__ inline short bf16_bits(double v) { return (short)to_bf16((float)v).bits; }

// The face-block Schur complement of one cell formed a second time, for the
// V-cycle's single-precision copy only: the FP64 factors already in LDS are
// rounded to bfloat16 and multiplied on the matrix cores (16x16x16 bfloat16
// products, FP32 accumulation); the outer operator keeps the FP64 product.
//   v-cond:   out = a_dd - W^T W                                   (m x m, K = nT)
//   v&p-cond: out = [c = c'] a_dd - sum_c [c = c'] W^T W + Z^T Z   (dm x dm)
// For v&p-cond one product runs over K = n1 + d nT: the n1 rows of Z, then the
// nT rows of W once per component, that part with a minus sign on the right
// factor and zero where the row's or column's component differs.  W[t][i] is
// W[t * ldw + i] (i a face unknown of one component), Z[t][row] is Z[t * dm + row].
// Wave w of the block takes the 16 x 16 output tiles w, w + nw, ...; out is the
// cell's n x n block, row-major.
__device__ void schur_product_bf16(int cond, int d, int nT, int nF, int nfc, const double *a, int nloc,
                                   const double *W, int ldw, const double *Z, int n1, float *out) {
  const int m = nfc * nF, dm = d * m;
  const int n = (cond == 1) ? m : dm;
  const int K = (cond == 1) ? nT : n1 + d * nT;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int nt = (n + 15) / 16, kt = (K + 15) / 16;
  // entry (row, k) of the left factor and (k, col) of the right one
  auto left = [&](int row, int k) -> double {
    if (cond == 1) return W[k * ldw + row];
    if (k < n1) return Z[k * dm + row];
    const int kk = k - n1, c = kk / nT, t = kk % nT;
    if ((row / nF) % d != c) return 0.0;
    return W[t * ldw + (row / (d * nF)) * nF + row % nF];
  };
  auto right = [&](int k, int col) -> double {
    if (cond == 1) return W[k * ldw + col];
    if (k < n1) return Z[k * dm + col];
    const int kk = k - n1, c = kk / nT, t = kk % nT;
    if ((col / nF) % d != c) return 0.0;
    return -W[t * ldw + (col / (d * nF)) * nF + col % nF];
  };
  for (int tile = wave; tile < nt * nt; tile += nw) {  // uniform over the wave: every lane takes part
    const int ti = tile / nt, tj = tile % nt;
    const int r = ti * 16 + lane % 16, c = tj * 16 + lane % 16;
    v4f32 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < kt; ++kb) {
      v4bf af, bf;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kb * 16 + 4 * (lane / 16) + v;
        af[v] = (r < n && k < K) ? bf16_bits(left(r, k)) : (short)0;
        bf[v] = (c < n && k < K) ? bf16_bits(right(k, c)) : (short)0;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = ti * 16 + 4 * (lane / 16) + v, col = c;
      if (row >= n || col >= n) continue;
      float base;
      if (cond == 1) {
        base = (float)a[(int64_t)(nT + row) * nloc + nT + col];
      } else {
        const int ci = (row / nF) % d, cj = (col / nF) % d;
        const int i = (row / (d * nF)) * nF + row % nF, j = (col / (d * nF)) * nF + col % nF;
        base = (ci == cj) ? (float)a[(int64_t)(nT + i) * nloc + nT + j] : 0.f;
      }
      // v-cond: the product is W^T W, subtracted; v&p: signs are in the factors
      out[(int64_t)row * n + col] = (cond == 1) ? base - acc[v] : base + acc[v];
    }
  }
}

// ------------------------------------------------------------ static condensation
// One block per cell.  Record of the cell (host-built, eq. def:HHOAB):
//   a [nloc][nloc] scalar viscous matrix (cell modes first, then faces),
//   B [d][nT][nloc] coupling per component, ru [d][nloc], rp [nT].
// With L the Cholesky factor of a_TT:
//   W = L^{-1} a_Td, Y_c = L^{-1} B_c,TT^T, g_c = L^{-1} f_c,
//   s = a_dd - W^T W                          (S_dd = s (x) I_d)
//   C_c = B_c,dT^T - W^T Y_c                  (S_dT)
//   S_TT = -sum_c Y_c^T Y_c
// (the Schur complement of eq. ST.1).  v&p-cond eliminates the non-mean pressure
// modes of this system as well (eq. ST.2): with Sigma = -S_TT[1:,1:] = L_s L_s^T
// and Z = L_s^{-1} C[:,1:]^T, S_dd^{vp} = s (x) I_d + Z^T Z and the coupling to
// the mean pressure is C[:,0].
__global__ void __launch_bounds__(kBlock) k_condense(DTopo tp, int cond, int nT, int nF, const double *rec,
                                                     const int64_t *roff, double *stage, double *cpl,
                                                     double *spp, double *rhs_stage, double *rhs_p, int *err,
                                                     float *stage32) {
  extern __shared__ double lds[];
  const int T = blockIdx.x;
  const int d = tp.d;
  const int nfc = tp.cptr[T + 1] - tp.cptr[T];
  const int m = nfc * nF;
  const int nloc = nT + m;
  const double *a = rec + roff[T];
  const double *B = a + (int64_t)nloc * nloc;
  const double *ru = B + (int64_t)d * nT * nloc;
  const double *rp = ru + (int64_t)d * nloc;
  // LDS: AT [nT][nloc] (L | W), Y [d][nT][nT], G [d][nT]
  double *AT = lds;
  double *Y = AT + nT * nloc;
  double *G = Y + d * nT * nT;
  double *ext = G + d * nT;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < nT * nloc; i += blockDim.x) AT[i] = a[i];
  for (int i = threadIdx.x; i < d * nT * nT; i += blockDim.x) {
    const int c = i / (nT * nT), t = (i / nT) % nT, q = i % nT;
    Y[i] = B[((int64_t)c * nT + q) * nloc + t];  // B_c,TT^T
  }
  for (int i = threadIdx.x; i < d * nT; i += blockDim.x) G[i] = ru[(i / nT) * nloc + i % nT];
  __syncthreads();
  blk_chol(AT, nT, nloc, &bad);
  __syncthreads();
  // W (in place, columns nT..nloc-1 of AT), Y_c (columns q), g_c
  blk_fwd(AT, nT, nloc, AT + nT, m, 1, nloc);
  for (int c = 0; c < d; ++c) blk_fwd(AT, nT, nloc, Y + c * nT * nT, nT, 1, nT);
  blk_fwd(AT, nT, nloc, G, d, nT, 1);
  __syncthreads();
  const double *W = AT + nT;  // W[t][j] = AT[t*nloc + nT + j]
  const int64_t c0 = tp.cptr[T];

  if (cond == 1) {
    double *s = stage + tp.pairoff[T] * nF * nF;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int i = idx / m, j = idx % m;
      double v = a[(int64_t)(nT + i) * nloc + nT + j];
      for (int t = 0; t < nT; ++t) v -= W[t * nloc + i] * W[t * nloc + j];
      s[idx] = v;
    }
    double *C = cpl + c0 * d * nF * nT;
    for (int idx = threadIdx.x; idx < d * m * nT; idx += blockDim.x) {
      const int row = idx / nT, q = idx % nT;
      const int fi = row / (d * nF), c = (row / nF) % d, r = row % nF;
      const int jl = fi * nF + r;
      double v = B[((int64_t)c * nT + q) * nloc + nT + jl];
      for (int t = 0; t < nT; ++t) v -= W[t * nloc + jl] * Y[(c * nT + t) * nT + q];
      C[idx] = v;
    }
    double *P = spp + (int64_t)T * nT * nT;
    for (int idx = threadIdx.x; idx < nT * nT; idx += blockDim.x) {
      const int q = idx / nT, q2 = idx % nT;
      double v = 0;
      for (int c = 0; c < d; ++c)
        for (int t = 0; t < nT; ++t) v -= Y[(c * nT + t) * nT + q] * Y[(c * nT + t) * nT + q2];
      P[idx] = v;
    }
    double *rs = rhs_stage + c0 * d * nF;
    for (int row = threadIdx.x; row < d * m; row += blockDim.x) {
      const int fi = row / (d * nF), c = (row / nF) % d, r = row % nF;
      const int jl = fi * nF + r;
      double v = ru[(int64_t)c * nloc + nT + jl];
      for (int t = 0; t < nT; ++t) v -= W[t * nloc + jl] * G[c * nT + t];
      rs[row] = v;
    }
    for (int q = threadIdx.x; q < nT; q += blockDim.x) {
      double v = rp[q];
      for (int c = 0; c < d; ++c)
        for (int t = 0; t < nT; ++t) v -= Y[(c * nT + t) * nT + q] * G[c * nT + t];
      rhs_p[(int64_t)T * nT + q] = v;
    }
    if (stage32)
      schur_product_bf16(cond, d, nT, nF, nfc, a, nloc, W, nloc, nullptr, 0,
                         stage32 + tp.pairoff[T] * nF * nF);
  } else {
    // ext: Ct [nT][d*m] (C transposed), Sg [(nT-1)^2], rP [nT], h [nT-1]
    const int dm = d * m, n1 = nT - 1;
    double *Ct = ext;
    double *Sg = Ct + nT * dm;
    double *rP = Sg + n1 * n1;
    double *h = rP + nT;
    for (int idx = threadIdx.x; idx < dm * nT; idx += blockDim.x) {
      const int row = idx / nT, q = idx % nT;
      const int fi = row / (d * nF), c = (row / nF) % d, r = row % nF;
      const int jl = fi * nF + r;
      double v = B[((int64_t)c * nT + q) * nloc + nT + jl];
      for (int t = 0; t < nT; ++t) v -= W[t * nloc + jl] * Y[(c * nT + t) * nT + q];
      Ct[q * dm + row] = v;
    }
    for (int idx = threadIdx.x; idx < n1 * n1; idx += blockDim.x) {
      const int q = 1 + idx / n1, q2 = 1 + idx % n1;
      double v = 0;
      for (int c = 0; c < d; ++c)
        for (int t = 0; t < nT; ++t) v += Y[(c * nT + t) * nT + q] * Y[(c * nT + t) * nT + q2];
      Sg[idx] = v;  // Sigma = -S_TT[1:,1:]
    }
    for (int q = threadIdx.x; q < nT; q += blockDim.x) {
      double v = rp[q];
      for (int c = 0; c < d; ++c)
        for (int t = 0; t < nT; ++t) v -= Y[(c * nT + t) * nT + q] * G[c * nT + t];
      rP[q] = v;
    }
    __syncthreads();
    if (n1 > 0) {
      blk_chol(Sg, n1, n1, &bad);
      __syncthreads();
      blk_fwd(Sg, n1, n1, Ct + dm, dm, 1, dm);      // Z = L_s^{-1} C[:,1:]^T (in place)
      for (int i = threadIdx.x; i < n1; i += blockDim.x) h[i] = rP[1 + i];
      __syncthreads();
      blk_fwd(Sg, n1, n1, h, 1, 1, 1);             // h = L_s^{-1} rhs_P~
      __syncthreads();
    }
    const double *Z = Ct + dm;
    double *S = stage + tp.pairoff[T] * (int64_t)(d * nF) * (d * nF);
    for (int idx = threadIdx.x; idx < dm * dm; idx += blockDim.x) {
      const int row = idx / dm, col = idx % dm;
      const int fi = row / (d * nF), c = (row / nF) % d, r = row % nF;
      const int fj = col / (d * nF), c2 = (col / nF) % d, r2 = col % nF;
      double v = 0;
      if (c == c2) {
        const int i = fi * nF + r, j = fj * nF + r2;
        v = a[(int64_t)(nT + i) * nloc + nT + j];
        for (int t = 0; t < nT; ++t) v -= W[t * nloc + i] * W[t * nloc + j];
      }
      for (int t = 0; t < n1; ++t) v += Z[t * dm + row] * Z[t * dm + col];
      S[idx] = v;
    }
    double *bb = cpl + c0 * d * nF;
    for (int row = threadIdx.x; row < dm; row += blockDim.x) bb[row] = Ct[row];
    double *rs = rhs_stage + c0 * d * nF;
    for (int row = threadIdx.x; row < dm; row += blockDim.x) {
      const int fi = row / (d * nF), c = (row / nF) % d, r = row % nF;
      const int jl = fi * nF + r;
      double v = ru[(int64_t)c * nloc + nT + jl];
      for (int t = 0; t < nT; ++t) v -= W[t * nloc + jl] * G[c * nT + t];
      // eliminate the non-mean pressure rows: r_d + C~ Sigma^{-1} r_P~
      for (int t = 0; t < n1; ++t) v += Z[t * dm + row] * h[t];
      rs[row] = v;
    }
    if (threadIdx.x == 0) rhs_p[T] = rP[0];
    if (stage32)
      schur_product_bf16(cond, d, nT, nF, nfc, a, nloc, W, nloc, Z, n1,
                         stage32 + tp.pairoff[T] * (int64_t)(d * nF) * (d * nF));
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicMax(err, T + 1);
}

// ------------------------------------------------------------ cell recovery
// Back-substitution of the eliminated cell unknowns from the solved globally
// coupled ones (Section 4.1.2), one block per cell, from the cell's record:
//  v-cond, first block row of eq. def:HHOAB:
//    a_TT U_T,c = f_c - a_Td U_dT,c - B_c,TT^T P_T.
//  v&p-cond, the eliminated block of eq. ST.2 with the mean pressure Pbar known:
//    r_c = f_c - a_Td U_dT,c - B_c,TT[0]^T Pbar,  s = rp[1:] - B~_d U_dT,
//    with L the Cholesky factor of a_TT, Y_c = L^{-1} B_c,TT^T, g_c = L^{-1} r_c
//    and Sigma = sum_c Y~_c^T Y~_c (non-mean columns), the non-mean pressures
//    solve Sigma P~ = sum_c Y~_c^T g_c - s and U_T,c = L^{-T} (g_c - Y~_c P~).
__global__ void __launch_bounds__(kBlock) k_recover(DTopo tp, int cond, int nT, int nF, const double *rec,
                                                    const int64_t *roff, const double *x, double *cu, double *cp,
                                                    int *err) {
  extern __shared__ double lds[];
  const int T = blockIdx.x;
  const int d = tp.d;
  const int64_t c0 = tp.cptr[T];
  const int nfc = tp.cptr[T + 1] - tp.cptr[T];
  const int m = nfc * nF, nloc = nT + m, n1 = nT - 1;
  const int np = (cond == 1) ? nT : 1;
  const double *a = rec + roff[T];
  const double *B = a + (int64_t)nloc * nloc;
  const double *ru = B + (int64_t)d * nT * nloc;
  const double *rp = ru + (int64_t)d * nloc;
  const double *xp = x + (int64_t)tp.nf * d * nF + (int64_t)T * np;
  // LDS: L [nT][nT], U [d][m] face unknowns per component, R [d][nT],
  //      p [nT] pressures, Y [d][nT][nT], Sg [n1][n1], h [nT]
  double *L = lds;
  double *U = L + nT * nT;
  double *R = U + d * m;
  double *p = R + d * nT;
  double *Y = p + nT;
  double *Sg = Y + d * nT * nT;
  double *h = Sg + n1 * n1;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < nT * nT; i += blockDim.x) L[i] = a[(int64_t)(i / nT) * nloc + i % nT];
  for (int i = threadIdx.x; i < d * m; i += blockDim.x) {
    const int c = i / m, j = i % m;
    const int f = tp.cface[c0 + j / nF];
    U[i] = x[((int64_t)f * d + c) * nF + j % nF];
  }
  for (int q = threadIdx.x; q < nT; q += blockDim.x) p[q] = (q < np) ? xp[q] : 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < d * nT; i += blockDim.x) {
    const int c = i / nT, t = i % nT;
    const double *at = a + (int64_t)t * nloc + nT;
    double v = ru[(int64_t)c * nloc + t];
    for (int j = 0; j < m; ++j) v -= at[j] * U[c * m + j];
    for (int q = 0; q < np; ++q) v -= B[((int64_t)c * nT + q) * nloc + t] * p[q];
    R[i] = v;
  }
  if (cond != 1) {
    for (int i = threadIdx.x; i < d * nT * nT; i += blockDim.x) {
      const int c = i / (nT * nT), t = (i / nT) % nT, q = i % nT;
      Y[i] = B[((int64_t)c * nT + q) * nloc + t];  // B_c,TT^T
    }
    for (int q = 1 + threadIdx.x; q < nT; q += blockDim.x) {
      double v = rp[q];
      for (int c = 0; c < d; ++c) {
        const double *bq = B + ((int64_t)c * nT + q) * nloc + nT;
        for (int j = 0; j < m; ++j) v -= bq[j] * U[c * m + j];
      }
      h[q] = v;
    }
  }
  __syncthreads();
  blk_chol(L, nT, nT, &bad);
  __syncthreads();
  blk_fwd(L, nT, nT, R, d, nT, 1);  // g_c
  if (cond != 1)
    for (int c = 0; c < d; ++c) blk_fwd(L, nT, nT, Y + c * nT * nT, nT, 1, nT);
  __syncthreads();
  if (cond != 1 && n1 > 0) {
    for (int idx = threadIdx.x; idx < n1 * n1; idx += blockDim.x) {
      const int q = 1 + idx / n1, q2 = 1 + idx % n1;
      double v = 0;
      for (int c = 0; c < d; ++c)
        for (int t = 0; t < nT; ++t) v += Y[(c * nT + t) * nT + q] * Y[(c * nT + t) * nT + q2];
      Sg[idx] = v;
    }
    for (int q = 1 + threadIdx.x; q < nT; q += blockDim.x) {
      double v = -h[q];
      for (int c = 0; c < d; ++c)
        for (int t = 0; t < nT; ++t) v += Y[(c * nT + t) * nT + q] * R[c * nT + t];
      p[q] = v;
    }
    __syncthreads();
    blk_chol(Sg, n1, n1, &bad);
    __syncthreads();
    blk_fwd(Sg, n1, n1, p + 1, 1, 1, 1);
    __syncthreads();
    blk_bwd(Sg, n1, n1, p + 1, 1, 1, 1);
    __syncthreads();
    for (int i = threadIdx.x; i < d * nT; i += blockDim.x) {
      const int c = i / nT, t = i % nT;
      double v = R[i];
      for (int q = 1; q < nT; ++q) v -= Y[(c * nT + t) * nT + q] * p[q];
      R[i] = v;
    }
    __syncthreads();
  }
  blk_bwd(L, nT, nT, R, d, nT, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < d * nT; i += blockDim.x) cu[(int64_t)T * d * nT + i] = R[i];
  for (int q = threadIdx.x; q < nT; q += blockDim.x) cp[(int64_t)T * nT + q] = p[q];
  if (threadIdx.x == 0 && bad) atomicMax(err, T + 1);
}

// ------------------------------------------------------------ assembly
// Every face block (F, F') is the sum of the <= 2 cell blocks (T, i, j) with
// F_i = F and F_j = F' (deterministic gather, no atomics).
__global__ void k_assemble(DTopo tp, int cond, int nF, int64_t nnzb, const double *stage, double *bsr) {
  const int d = tp.d;
  const int bs = (cond == 1) ? nF : d * nF;
  const int64_t total = nnzb * bs * bs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / (bs * bs);
    const int rr = (int)(e % (bs * bs)) / bs, cc = (int)(e % bs);
    double v = 0;
    for (int s = 0; s < 2; ++s) {
      const int T = tp.blksrc[6 * b + 3 * s];
      if (T < 0) continue;
      const int i = tp.blksrc[6 * b + 3 * s + 1], j = tp.blksrc[6 * b + 3 * s + 2];
      const int nfc = tp.cptr[T + 1] - tp.cptr[T];
      const int64_t dim = (int64_t)nfc * bs;
      const double *S = stage + tp.pairoff[T] * bs * bs;
      v += S[(i * bs + rr) * dim + j * bs + cc];
    }
    bsr[e] = v;
  }
}

// The same gather for the V-cycle's copy: FP32 cell blocks summed in FP32 and
// stored as Tout (float or bf16).
template <typename Tout>
__global__ void k_assemble32(DTopo tp, int cond, int nF, int64_t nnzb, const float *stage, Tout *bsr) {
  const int d = tp.d;
  const int bs = (cond == 1) ? nF : d * nF;
  const int64_t total = nnzb * bs * bs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / (bs * bs);
    const int rr = (int)(e % (bs * bs)) / bs, cc = (int)(e % bs);
    float v = 0;
    for (int s = 0; s < 2; ++s) {
      const int T = tp.blksrc[6 * b + 3 * s];
      if (T < 0) continue;
      const int i = tp.blksrc[6 * b + 3 * s + 1], j = tp.blksrc[6 * b + 3 * s + 2];
      const int nfc = tp.cptr[T + 1] - tp.cptr[T];
      const int64_t dim = (int64_t)nfc * bs;
      const float *S = stage + tp.pairoff[T] * bs * bs;
      v += S[(i * bs + rr) * dim + j * bs + cc];
    }
    bsr[e] = StoreAs<Tout>::from(v);
  }
}

// Face part of the condensed right-hand side: sum of the two cells' contributions.
__global__ void k_rhs_faces(DTopo tp, int nF, const double *rhs_stage, double *rhs) {
  const int d = tp.d;
  const int64_t total = (int64_t)tp.nf * d * nF;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(e / (d * nF));
    const int cr = (int)(e % (d * nF));
    double v = 0;
    for (int s = 0; s < 2; ++s) {
      const int T = tp.fcell[2 * f + s];
      if (T < 0) continue;
      v += rhs_stage[((int64_t)tp.cptr[T] + tp.floc[2 * f + s]) * d * nF + cr];
    }
    rhs[e] = v;
  }
}

// ------------------------------------------------------------ level inheritance
// S^{l+1} = I S^l I^T with unit-diagonal restriction: keep the leading face
// modes of every block and the leading pressure modes of every cell.
__global__ void k_extract(DTopo tp, int cond, int64_t nnzb, int p0, int t0, int p1, int t1, const double *bsr0,
                          const double *cpl0, const double *spp0, double *bsr1, double *cpl1, double *spp1) {
  const int d = tp.d;
  const int b0 = (cond == 1) ? p0 : d * p0, b1 = (cond == 1) ? p1 : d * p1;
  const int64_t nb = nnzb * b1 * b1;
  const int64_t ncpl = (cond == 1) ? tp.ncf * d * p1 * t1 : tp.ncf * d * p1;
  const int64_t nspp = (cond == 1) ? (int64_t)tp.nc * t1 * t1 : 0;
  const int64_t total = nb + ncpl + nspp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nb) {
      const int64_t b = e / (b1 * b1);
      const int rr = (int)(e % (b1 * b1)) / b1, cc = (int)(e % b1);
      int r0 = rr, c0 = cc;
      if (cond != 1) {
        r0 = (rr / p1) * p0 + rr % p1;
        c0 = (cc / p1) * p0 + cc % p1;
      }
      bsr1[e] = bsr0[b * b0 * b0 + (int64_t)r0 * b0 + c0];
    } else if (e < nb + ncpl) {
      const int64_t x = e - nb;
      if (cond == 1) {
        const int64_t row = x / t1;  // (entry, c, r) with r < p1
        const int q = (int)(x % t1);
        const int64_t ec = row / p1;
        const int r = (int)(row % p1);
        cpl1[x] = cpl0[(ec * p0 + r) * t0 + q];
      } else {
        const int64_t ec = x / p1;
        const int r = (int)(x % p1);
        cpl1[x] = cpl0[ec * p0 + r];
      }
    } else {
      const int64_t x = e - nb - ncpl;
      const int64_t T = x / (t1 * t1);
      const int q = (int)(x % (t1 * t1)) / t1, q2 = (int)(x % t1);
      spp1[x] = spp0[T * t0 * t0 + (int64_t)q * t0 + q2];
    }
  }
}

// ------------------------------------------------------------ smoother patches
// Patch of cell T = the unknowns of its faces and its pressure; the patch matrix
// is the level operator restricted to it.
//  v-cond: [[s_P (x) I_d, C], [C^T, S_TT]]: store s_P^{-1} and the inverse of the
//          pressure Schur complement X = S_TT - C^T (s_P^{-1} (x) I_d) C.
//  v&p:    [[S_P, b], [b^T, 0]]: store S_P^{-1}, g = S_P^{-1} b, 1/(b^T g).
// The symmetric inverses are stored as their lower triangle packed by rows
// (entry (i, j), i >= j, at i (i + 1) / 2 + j) at the start of the cell's slot.
// The factor is formed in `scratch` (per-cell slots sized like s_P).
__global__ void __launch_bounds__(kBlock) k_patch_setup(DTopo tp, int cond, int p, int t, const double *bsr,
                                                        const double *cpl, const double *spp, double *sinv,
                                                        double *xinv, double *sig, double *scratch, int *err) {
  extern __shared__ double lds[];
  const int T = blockIdx.x;
  const int d = tp.d;
  const int nfc = tp.cptr[T + 1] - tp.cptr[T];
  const int bs = (cond == 1) ? p : d * p;  // block edge
  const int n = nfc * bs;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  double *Lm = scratch + tp.pairoff[T] * bs * bs;
  double *Si = sinv + tp.pairoff[T] * bs * bs;
  const int32_t *pb = tp.pairblk + tp.pairoff[T];
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    const int fi = i / bs, fj = j / bs;
    const int64_t blk = pb[fi * nfc + fj];
    Lm[idx] = bsr[blk * bs * bs + (int64_t)(i % bs) * bs + (j % bs)];
  }
  __syncthreads();
  blk_chol(Lm, n, n, &bad);
  __syncthreads();
  blk_chol_inverse(Lm, n, n, Si, n);
  const int64_t c0 = tp.cptr[T];
  if (cond == 1) {
    // U = (s^{-1} (x) I) C  [d*n x t], X = S_TT - C^T U  [t x t]
    const double *C = cpl + c0 * d * p * t;
    double *U = lds;              // [d*n][t]
    double *X = U + d * n * t;    // [t][t]
    for (int idx = threadIdx.x; idx < d * n * t; idx += blockDim.x) {
      const int row = idx / t, q = idx % t;
      const int fi = row / (d * p), c = (row / p) % d, r = row % p;
      const int i = fi * p + r;
      double v = 0;
      for (int fj = 0; fj < nfc; ++fj)
        for (int r2 = 0; r2 < p; ++r2) v += Si[i * n + fj * p + r2] * C[((fj * d + c) * p + r2) * t + q];
      U[idx] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) {
      const int q = idx / t, q2 = idx % t;
      double v = -spp[(int64_t)T * t * t + idx];
      for (int row = 0; row < d * n; ++row) v += C[row * t + q] * U[row * t + q2];
      X[idx] = v;  // -X is SPD
    }
    __syncthreads();
    blk_chol(X, t, t, &bad);
    __syncthreads();
    double *Xi = xinv + (int64_t)T * t * t;
    blk_chol_inverse(X, t, t, Xi, t);
    for (int idx = threadIdx.x; idx < t * t; idx += blockDim.x) Xi[idx] = -Xi[idx];
  } else {
    const double *b = cpl + c0 * d * p;
    double *g = xinv + c0 * d * p;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      double v = 0;
      for (int j = 0; j < n; ++j) v += Si[i * n + j] * b[j];
      g[i] = v;
    }
    __syncthreads();
    double part = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) part += b[i] * g[i];
    const double s = block_sum(part, lds);
    if (threadIdx.x == 0) {
      if (!(s > 0.0)) bad = 1;
      sig[T] = (s > 0.0) ? 1.0 / s : 0.0;
    }
  }
  // keep S_P^{-1} as its lower triangle packed by rows (through a copy in the scratch slot)
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) Lm[idx] = Si[idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    if (j <= i) Si[(int64_t)i * (i + 1) / 2 + j] = Lm[idx];
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicMax(err, T + 1);
}

// Same outputs as k_patch_setup with the patch factorised entirely in LDS:
// the lower triangle of the patch matrix is held packed by columns
// (n(n+1)/2 doubles, 130 KB for n = 180), factorised in place (Cholesky), and
// the factor inverted in place (L^{-1}); S_P^{-1} = L^{-T} L^{-1} is formed
// entry by entry straight into global memory.  One 512-thread block per cell;
// waves take columns, lanes run down a column (consecutive LDS addresses).
constexpr int kPatchThreads = 512;

__device__ inline int pk(int n, int i, int j) { return j * (2 * n - j + 1) / 2 + (i - j); }  // i >= j

__global__ void __launch_bounds__(kPatchThreads) k_patch_setup_lds(DTopo tp, int cond, int p, int t,
                                                                   const double *bsr, const double *cpl,
                                                                   const double *spp, double *sinv, double *xinv,
                                                                   double *sig, int *err) {
  extern __shared__ double lds[];
  const int T = blockIdx.x;
  const int d = tp.d;
  const int nfc = tp.cptr[T + 1] - tp.cptr[T];
  const int bs = (cond == 1) ? p : d * p;
  const int n = nfc * bs;
  const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave, nw = blockDim.x / kWave;
  double *A = lds;                       // packed lower, n(n+1)/2
  double *x = A + n * (n + 1) / 2;       // [max(n, 16)] scratch column / reduction space
  double *ext = x + (n > 16 ? n : 16);   // v-cond: U [d*n][t], X [t][t], 2 columns; v&p: [n]
  __shared__ int bad;
  if (tid == 0) bad = 0;
  const int32_t *pb = tp.pairblk + tp.pairoff[T];
  for (int j = wid; j < n; j += nw)
    for (int i = j + lane; i < n; i += kWave) {
      const int fi = i / bs, fj = j / bs;
      const int64_t blk = pb[fi * nfc + fj];
      A[pk(n, i, j)] = bsr[blk * bs * bs + (int64_t)(i % bs) * bs + (j % bs)];
    }
  __syncthreads();
  // Cholesky, right-looking
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      double v = A[pk(n, j, j)];
      if (!(v > 0.0)) {
        bad = 1;
        v = 1.0;
      }
      A[pk(n, j, j)] = sqrt(v);
    }
    __syncthreads();
    const double ljj = A[pk(n, j, j)];
    for (int i = j + 1 + tid; i < n; i += blockDim.x) A[pk(n, i, j)] /= ljj;
    __syncthreads();
    for (int k = j + 1 + wid; k < n; k += nw) {
      const double akj = A[pk(n, k, j)];
      double *ck = A + pk(n, k, k);
      const double *cj = A + pk(n, k, j);
      for (int i = lane; i < n - k; i += kWave) ck[i] -= cj[i] * akj;
    }
    __syncthreads();
  }
  // L^{-1} in place, last column first: column j below the diagonal becomes
  // -L^{-1}_jj * (L^{-1})_{trailing} * L_{j+1:, j}; one wave per row, lanes split
  // the row's dot product (fixed-order wave reduction)
  for (int j = n - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < n; i += blockDim.x) x[i] = A[pk(n, i, j)];
    if (tid == 0) A[pk(n, j, j)] = 1.0 / A[pk(n, j, j)];
    __syncthreads();
    const double ajj = A[pk(n, j, j)];
    for (int i = j + 1 + wid; i < n; i += nw) {
      double acc = 0;
      for (int k = j + 1 + lane; k <= i; k += kWave) acc += A[pk(n, i, k)] * x[k];
      acc = wave_sum(acc);
      if (lane == 0) A[pk(n, i, j)] = -ajj * acc;
    }
    __syncthreads();
  }
  // S_P^{-1}(i, k) = sum_{m >= max(i,k)} Linv(m, i) Linv(m, k), lower triangle packed by rows
  double *Si = sinv + tp.pairoff[T] * (int64_t)bs * bs;
  for (int k = wid; k < n; k += nw)
    for (int i = k + lane; i < n; i += kWave) {
      double acc = 0;
      const double *ci = A + pk(n, i, i), *ck = A + pk(n, i, k);  // rows m >= i of columns i and k
      for (int m = 0; m < n - i; ++m) acc += ci[m] * ck[m];
      Si[(int64_t)i * (i + 1) / 2 + k] = acc;
    }
  // y = S_P^{-1} v through the factor: u = Linv v, y = Linv^T u (columns of V strided by ld)
  auto apply = [&](const double *v, int64_t vs, double *u, double *y, int64_t ys) {
    for (int i = tid; i < n; i += blockDim.x) {
      double acc = 0;
      for (int k = 0; k <= i; ++k) acc += A[pk(n, i, k)] * v[k * vs];
      u[i] = acc;
    }
    __syncthreads();
    for (int k = tid; k < n; k += blockDim.x) {
      double acc = 0;
      const double *ck = A + pk(n, k, k);
      for (int m = 0; m < n - k; ++m) acc += ck[m] * u[k + m];
      y[k * ys] = acc;
    }
    __syncthreads();
  };
  const int64_t c0 = tp.cptr[T];
  if (cond == 1) {
    // U = (s^{-1} (x) I) C  [(face, comp, mode) x t], X = S_TT - C^T U  [t x t]
    const double *C = cpl + c0 * d * p * t;
    double *U = ext;                      // [nfc*d*p][t]
    double *X = U + (int64_t)d * n * t;   // [t][t]
    double *vcol = X + t * t;             // [n]
    double *ycol = vcol + n;              // [n]
    for (int c = 0; c < d; ++c)
      for (int q = 0; q < t; ++q) {
        for (int i = tid; i < n; i += blockDim.x) {
          const int fj = i / p, r = i % p;
          vcol[i] = C[((fj * d + c) * p + r) * t + q];
        }
        __syncthreads();
        apply(vcol, 1, x, ycol, 1);
        for (int i = tid; i < n; i += blockDim.x) {
          const int fj = i / p, r = i % p;
          U[((fj * d + c) * p + r) * t + q] = ycol[i];
        }
        __syncthreads();
      }
    for (int idx = tid; idx < t * t; idx += blockDim.x) {
      const int q = idx / t, q2 = idx % t;
      double v = -spp[(int64_t)T * t * t + idx];
      for (int row = 0; row < d * n; ++row) v += C[row * t + q] * U[row * t + q2];
      X[idx] = v;  // -X is SPD
    }
    __syncthreads();
    blk_chol(X, t, t, &bad);
    __syncthreads();
    double *Xi = xinv + (int64_t)T * t * t;
    blk_chol_inverse(X, t, t, Xi, t);
    for (int idx = tid; idx < t * t; idx += blockDim.x) Xi[idx] = -Xi[idx];
  } else {
    const double *b = cpl + c0 * d * p;
    double *g = xinv + c0 * d * p;
    double *gl = ext;  // [n]
    apply(b, 1, x, gl, 1);
    double part = 0;
    for (int i = tid; i < n; i += blockDim.x) {
      g[i] = gl[i];
      part += b[i] * gl[i];
    }
    __syncthreads();
    const double sdot = block_sum(part, x);
    if (tid == 0) {
      if (!(sdot > 0.0)) bad = 1;
      sig[T] = (sdot > 0.0) ? 1.0 / sdot : 0.0;
    }
  }
  __syncthreads();
  if (tid == 0 && bad) atomicMax(err, T + 1);
}

// Patch inverse by the sweep operator (Gauss-Jordan elimination in place on a
// symmetric positive definite matrix, pivots in order, no pivoting): sweeping
// pivot k maps a_kk -> -1/a_kk, a_ik -> a_ik/a_kk, a_kj -> a_kj/a_kk and
// a_ij -> a_ij - a_ik a_kj / a_kk; after all pivots the matrix is -S_P^{-1}.
// The pivots are the diagonal entries of the successive Schur complements,
// positive for an SPD patch.  The matrix lives in registers: thread t owns the
// TILE x TILE tile (t / nt, t % nt) (nt = ceil(n / TILE) tiles a side); the
// pivot column is broadcast through LDS (two barriers per pivot).  Padding rows
// and columns (n..nt*TILE) never couple to the patch.
template <int TILE>
__global__ void __launch_bounds__(1024) k_patch_sweep(DTopo tp, int cond, int p, int t, const double *bsr,
                                                      const double *cpl, const double *spp, double *sinv,
                                                      double *xinv, double *sig, int *err) {
  extern __shared__ double lds[];
  const int T = blockIdx.x;
  const int d = tp.d;
  const int nfc = tp.cptr[T + 1] - tp.cptr[T];
  const int bs = (cond == 1) ? p : d * p;
  const int n = nfc * bs;
  const int nt = (n + TILE - 1) / TILE;
  const int np = nt * TILE;
  const int tid = threadIdx.x;
  const int tr = tid / nt, tc = tid % nt;
  const bool own = tr < nt;
  const int r0 = tr * TILE, c0 = tc * TILE;
  // two pivot-column buffers [np + 1] (entry np: the pivot's reciprocal), used
  // alternately so that one barrier per pivot suffices
  const int cbw = np + 1;
  double *cbuf = lds;
  double *ext = cbuf + (2 * cbw > 16 ? 2 * cbw : 16);  // post-processing space
  __shared__ int bad;
  if (tid == 0) bad = 0;
  const int32_t *pb = tp.pairblk + tp.pairoff[T];
  double a[TILE][TILE];
#pragma unroll
  for (int q = 0; q < TILE; ++q)
#pragma unroll
    for (int w = 0; w < TILE; ++w) {
      const int i = r0 + q, j = c0 + w;
      double v = (i == j) ? 1.0 : 0.0;  // identity on the padding
      if (own && i < n && j < n) {
        const int64_t blk = pb[(i / bs) * nfc + (j / bs)];
        v = bsr[blk * bs * bs + (int64_t)(i % bs) * bs + (j % bs)];
      }
      a[q][w] = v;
    }
  // pivots k = kt TILE + W: the inner loop over W is unrolled, so the pivot's
  // place inside a tile is a compile-time index (direct register accesses, no
  // per-entry selects)
  for (int kt = 0; kt * TILE < n; ++kt) {
#pragma unroll
    for (int W = 0; W < TILE; ++W) {
      const int k = kt * TILE + W;
      if (k >= n) break;  // uniform
      double *cb = cbuf + (k & 1) * cbw;
      if (own && tc == kt) {
#pragma unroll
        for (int q = 0; q < TILE; ++q) cb[r0 + q] = a[q][W];
        if (tr == kt) {  // the diagonal's owner: the reciprocal, once
          const double dk = a[W][W];
          if (!(dk > 0.0)) bad = 1;
          cb[np] = (dk > 0.0) ? 1.0 / dk : 1.0;
        }
      }
      __syncthreads();
      const double inv = cb[np];
      if (own) {
        double ci[TILE], cj[TILE];
#pragma unroll
        for (int q = 0; q < TILE; ++q) {
          ci[q] = cb[r0 + q] * inv;
          cj[q] = cb[c0 + q];
        }
        // every entry: a_ij -= (a_ik / a_kk) a_kj (one FMA); the pivot row and
        // column, held by one tile row and one tile column, are fixed up after
#pragma unroll
        for (int q = 0; q < TILE; ++q)
#pragma unroll
          for (int w = 0; w < TILE; ++w) a[q][w] = fma(-ci[q], cj[w], a[q][w]);
        if (tr == kt) {
#pragma unroll
          for (int w = 0; w < TILE; ++w) a[W][w] = cj[w] * inv;
        }
        if (tc == kt) {
#pragma unroll
          for (int q = 0; q < TILE; ++q) a[q][W] = ci[q];
          if (tr == kt) a[W][W] = -inv;
        }
      }
      // no second barrier: the next pivot writes the other column buffer, and
      // every thread has read this one before it passes the next pivot's barrier
    }
  }
  __syncthreads();
  // S_P^{-1} = -a
  double *Si = sinv + tp.pairoff[T] * (int64_t)bs * bs;
  if (own) {
#pragma unroll
    for (int q = 0; q < TILE; ++q)
#pragma unroll
      for (int w = 0; w < TILE; ++w) {
        const int i = r0 + q, j = c0 + w;
        if (i < n && j <= i) Si[(int64_t)i * (i + 1) / 2 + j] = -a[q][w];
      }
  }
  const int64_t c0e = tp.cptr[T];
  if (cond == 1) {
    // the inverse in LDS (full square), then U = (s^{-1} (x) I) C and the pressure Schur complement
    double *Sl = ext;                        // [n][n]
    double *U = Sl + n * n;                  // [d*n][t]
    double *X = U + (int64_t)d * n * t;      // [t][t]
    if (own) {
#pragma unroll
      for (int q = 0; q < TILE; ++q)
#pragma unroll
        for (int w = 0; w < TILE; ++w) {
          const int i = r0 + q, j = c0 + w;
          if (i < n && j < n) Sl[i * n + j] = -a[q][w];
        }
    }
    __syncthreads();
    const double *C = cpl + c0e * d * p * t;
    for (int idx = tid; idx < d * n * t; idx += blockDim.x) {
      const int row = idx / t, q = idx % t;
      const int fi = row / (d * p), c = (row / p) % d, r = row % p;
      const int i = fi * p + r;
      double v = 0;
      for (int fj = 0; fj < nfc; ++fj)
        for (int r2 = 0; r2 < p; ++r2) v += Sl[i * n + fj * p + r2] * C[((fj * d + c) * p + r2) * t + q];
      U[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < t * t; idx += blockDim.x) {
      const int q = idx / t, q2 = idx % t;
      double v = -spp[(int64_t)T * t * t + idx];
      for (int row = 0; row < d * n; ++row) v += C[row * t + q] * U[row * t + q2];
      X[idx] = v;  // -X is SPD
    }
    __syncthreads();
    blk_chol(X, t, t, &bad);
    __syncthreads();
    double *Xi = xinv + (int64_t)T * t * t;
    blk_chol_inverse(X, t, t, Xi, t);
    for (int idx = tid; idx < t * t; idx += blockDim.x) Xi[idx] = -Xi[idx];
  } else {
    // g = S_P^{-1} b: per-tile partial row sums, then summed over tile columns in order
    const double *b = cpl + c0e * d * p;
    double *part = ext;                      // [nt][np]
    double *g = xinv + c0e * d * p;
    if (own) {
#pragma unroll
      for (int q = 0; q < TILE; ++q) {
        double sacc = 0;
#pragma unroll
        for (int w = 0; w < TILE; ++w)
          if (c0 + w < n) sacc -= a[q][w] * b[c0 + w];
        part[tc * np + r0 + q] = sacc;
      }
    }
    __syncthreads();
    double dot = 0;
    for (int i = tid; i < n; i += blockDim.x) {
      double gi = 0;
      for (int c = 0; c < nt; ++c) gi += part[c * np + i];
      g[i] = gi;
      dot += b[i] * gi;
    }
    __syncthreads();
    const double sdot = block_sum(dot, cbuf);
    if (tid == 0) {
      if (!(sdot > 0.0)) bad = 1;
      sig[T] = (sdot > 0.0) ? 1.0 / sdot : 0.0;
    }
  }
  __syncthreads();
  if (tid == 0 && bad) atomicMax(err, T + 1);
}

size_t patch_sweep_lds_bytes(int d, int cond, int p, int t, int max_faces, int tile) {
  const int64_t n = (int64_t)max_faces * ((cond == 1) ? p : d * p);
  const int64_t nt = (n + tile - 1) / tile;
  int64_t w = std::max<int64_t>(2 * (nt * tile + 1), 16);  // two pivot-column buffers
  w += (cond == 1) ? n * n + (int64_t)d * n * t + (int64_t)t * t : nt * nt * tile;
  return (size_t)w * sizeof(double);
}

template <typename Tout, typename Tin>
__global__ void k_convert(const Tin *in, Tout *out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = StoreAs<Tout>::from(in[i]);
}

// ------------------------------------------------------------ dense coarse level
// D = coarsest operator as a dense matrix, bordered by the constant-pressure
// vector when the operator is singular (row/col N).
__global__ void k_densify(DTopo tp, DLevel<double> L, int border, double *D, int64_t ld) {
  const int d = tp.d, p = L.p, t = L.t;
  const int bs = (L.cond == 1) ? p : d * p;
  const int64_t nb = tp.nnzb * bs * bs;
  const int64_t ncpl = tp.ncf * d * p * t;
  const int64_t nspp = (L.cond == 1) ? (int64_t)tp.nc * t * t : 0;
  const int64_t nbord = border ? (int64_t)tp.nc : 0;
  const int64_t total = nb + ncpl + nspp + nbord;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nb) {
      const int64_t b = e / (bs * bs);
      const int rr = (int)(e % (bs * bs)) / bs, cc = (int)(e % bs);
      // row face: binary search of b in rowptr
      int lo = 0, hi = tp.nf;
      while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (tp.rowptr[mid] <= b) lo = mid; else hi = mid;
      }
      const int f = lo, g = tp.col[b];
      if (L.cond == 1) {
        for (int c = 0; c < d; ++c) D[((int64_t)(f * d + c) * p + rr) * ld + (int64_t)(g * d + c) * p + cc] = L.bsr[e];
      } else {
        D[((int64_t)f * bs + rr) * ld + (int64_t)g * bs + cc] = L.bsr[e];
      }
    } else if (e < nb + ncpl) {
      const int64_t x = e - nb;
      const int64_t row = x / t;
      const int q = (int)(x % t);
      const int64_t ent = row / (d * p);  // cell-face entry
      const int cr = (int)(row % (d * p));
      // owning cell of the entry: binary search in cptr
      int lo = 0, hi = tp.nc;
      while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (tp.cptr[mid] <= ent) lo = mid; else hi = mid;
      }
      const int T = lo, f = tp.cface[ent];
      const int64_t rf = (int64_t)f * d * p + cr, cT = L.nface + (int64_t)T * t + q;
      D[rf * ld + cT] = L.cpl[x];
      D[cT * ld + rf] = L.cpl[x];
    } else if (e < nb + ncpl + nspp) {
      const int64_t x = e - nb - ncpl;
      const int64_t T = x / (t * t);
      const int q = (int)(x % (t * t)) / t, q2 = (int)(x % t);
      D[(L.nface + T * t + q) * ld + L.nface + T * t + q2] = L.spp[x];
    } else {
      const int64_t T = e - nb - ncpl - nspp;
      const int64_t N = L.N;
      D[N * ld + L.nface + T * t] = tp.zmean[T];
      D[(L.nface + T * t) * ld + N] = tp.zmean[T];
    }
  }
}

__global__ void k_eye_right(double *D, int64_t n, int64_t ld) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    D[i * ld + n + i] = 1.0;
}

// One Gauss-Jordan step with partial pivoting on the augmented [D | I]
// (n rows, 2n columns).  Phase 0 (one block): pivot search, row swap, scaling,
// copy of column k to colbuf.  Phase 1 (grid): elimination of column k.
__global__ void k_gj_pivot(double *D, int64_t n, int64_t ld, int64_t k, double *colbuf, int *err) {
  __shared__ double sv[kBlock];
  __shared__ int64_t si[kBlock];
  double best = -1;
  int64_t bi = k;
  for (int64_t i = k + threadIdx.x; i < n; i += blockDim.x) {
    double v = fabs(D[i * ld + k]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      if (sv[threadIdx.x + o] > sv[threadIdx.x] ||
          (sv[threadIdx.x + o] == sv[threadIdx.x] && si[threadIdx.x + o] < si[threadIdx.x])) {
        sv[threadIdx.x] = sv[threadIdx.x + o];
        si[threadIdx.x] = si[threadIdx.x + o];
      }
    }
    __syncthreads();
  }
  const int64_t piv = si[0];
  if (!(sv[0] > 0.0)) {
    if (threadIdx.x == 0) *err = 1;
    return;
  }
  if (piv != k)
    for (int64_t j = threadIdx.x; j < 2 * n; j += blockDim.x) {
      double a = D[k * ld + j];
      D[k * ld + j] = D[piv * ld + j];
      D[piv * ld + j] = a;
    }
  __syncthreads();
  const double inv = 1.0 / D[k * ld + k];
  __syncthreads();
  for (int64_t j = threadIdx.x; j < 2 * n; j += blockDim.x) D[k * ld + j] *= inv;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) colbuf[i] = (i == k) ? 0.0 : D[i * ld + k];
}

__global__ void k_gj_elim(double *D, int64_t n, int64_t ld, int64_t k, const double *colbuf) {
  const int64_t total = n * 2 * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / (2 * n), j = e % (2 * n);
    if (i == k) continue;
    const double f = colbuf[i];
    if (f != 0.0) D[i * ld + j] -= f * D[k * ld + j];
  }
}

// y = Dinv [x ; 0] (the border unknown is dropped), one wave per row.
__global__ void k_dense_matvec(const double *Dinv, int64_t n, int64_t ld, int border, const double *x,
                               double *y) {
  const int lane = threadIdx.x % kWave;
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t N = border ? n - 1 : n;
  if (row >= N) return;
  const double *R = Dinv + row * ld + n;  // inverse stored in the right half
  double v = 0;
  for (int64_t j = lane; j < N; j += kWave) v += R[j] * x[j];
  v = wave_sum(v);
  if (lane == 0) y[row] = v;
}

inline int grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65535 * 4) g = 65535 * 4;
  return (int)g;
}

}  // namespace

// ------------------------------------------------------------ launch wrappers
size_t condense_lds_bytes(int d, int cond, int nT, int nF, int max_faces) {
  const int m = max_faces * nF, nloc = nT + m;
  size_t n = (size_t)nT * nloc + (size_t)d * nT * nT + (size_t)d * nT;
  if (cond != 1) n += (size_t)nT * d * m + (size_t)(nT - 1) * (nT - 1) + nT + nT;
  return n * sizeof(double);
}
size_t patch_lds_bytes(int d, int cond, int p, int t, int max_faces) {
  const int n = max_faces * ((cond == 1) ? p : d * p);
  size_t x = (cond == 1) ? (size_t)d * n * t + (size_t)t * t : 16;
  return std::max<size_t>(x, 16) * sizeof(double);
}

void launch_condense(const DTopo &tp, int cond, int nT, int nF, const double *rec, const int64_t *roff,
                     double *stage, double *cpl, double *spp, double *rhs_stage, double *rhs_p, int *err,
                     hipStream_t s, size_t lds, float *stage32) {
  hipLaunchKernelGGL(k_condense, dim3(tp.nc), dim3(kBlock), lds, s, tp, cond, nT, nF, rec, roff, stage, cpl, spp,
                     rhs_stage, rhs_p, err, stage32);
}
template <typename Tout>
void launch_assemble32(const DTopo &tp, int cond, int nF, int64_t nnzb, const float *stage32, Tout *bsr,
                       hipStream_t s) {
  const int bs = (cond == 1) ? nF : tp.d * nF;
  hipLaunchKernelGGL((k_assemble32<Tout>), dim3(grid_for(nnzb * bs * bs)), dim3(kBlock), 0, s, tp, cond, nF, nnzb,
                     stage32, bsr);
}
template void launch_assemble32<float>(const DTopo &, int, int, int64_t, const float *, float *, hipStream_t);
template void launch_assemble32<bf16>(const DTopo &, int, int, int64_t, const float *, bf16 *, hipStream_t);
size_t recover_lds_bytes(int d, int nT, int nF, int max_faces) {
  const int m = max_faces * nF;
  const size_t n = (size_t)nT * nT + (size_t)d * m + (size_t)d * nT + nT + (size_t)d * nT * nT +
                   (size_t)(nT - 1) * (nT - 1) + nT;
  return n * sizeof(double);
}
void launch_recover(const DTopo &tp, int cond, int nT, int nF, const double *rec, const int64_t *roff,
                    const double *x, double *cu, double *cp, int *err, hipStream_t s, size_t lds) {
  if (tp.nc == 0) return;
  hipLaunchKernelGGL(k_recover, dim3(tp.nc), dim3(kBlock), lds, s, tp, cond, nT, nF, rec, roff, x, cu, cp, err);
}
void launch_assemble(const DTopo &tp, int cond, int nF, int64_t nnzb, const double *stage, double *bsr,
                     const double *rhs_stage, double *rhs, hipStream_t s) {
  const int bs = (cond == 1) ? nF : tp.d * nF;
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(nnzb * bs * bs)), dim3(kBlock), 0, s, tp, cond, nF, nnzb, stage, bsr);
  hipLaunchKernelGGL(k_rhs_faces, dim3(grid_for((int64_t)tp.nf * tp.d * nF)), dim3(kBlock), 0, s, tp, nF, rhs_stage,
                     rhs);
}
void launch_extract(const DTopo &tp, int cond, int64_t nnzb, int p0, int t0, int p1, int t1, const double *bsr0,
                    const double *cpl0, const double *spp0, double *bsr1, double *cpl1, double *spp1,
                    hipStream_t s) {
  const int b1 = (cond == 1) ? p1 : tp.d * p1;
  int64_t total = nnzb * b1 * b1 + tp.ncf * tp.d * p1 * ((cond == 1) ? t1 : 1) +
                  ((cond == 1) ? (int64_t)tp.nc * t1 * t1 : 0);
  hipLaunchKernelGGL(k_extract, dim3(grid_for(total)), dim3(kBlock), 0, s, tp, cond, nnzb, p0, t0, p1, t1, bsr0,
                     cpl0, spp0, bsr1, cpl1, spp1);
}
size_t patch_lds_packed_bytes(int d, int cond, int p, int t, int max_faces) {
  const int64_t n = (int64_t)max_faces * ((cond == 1) ? p : d * p);
  int64_t w = n * (n + 1) / 2 + std::max<int64_t>(n, 16);
  w += (cond == 1) ? (int64_t)d * n * t + (int64_t)t * t + 2 * n : n;
  return (size_t)std::max<int64_t>(w, 64) * sizeof(double);
}

void launch_patch_setup(const DTopo &tp, int cond, int p, int t, const double *bsr, const double *cpl,
                        const double *spp, double *sinv, double *xinv, double *sig, double *scratch, int *err,
                        hipStream_t s, size_t lds, int threads) {
  // register-resident sweep when a tile of at most 7 x 7 per thread covers the patch
  {
    const int n = tp.max_faces * ((cond == 1) ? p : tp.d * p);
    // one wavefront (8 x 8 tiles of at most 7 x 7) when the patch fits, so the
    // two barriers per pivot are cheap; else 32 x 32 tiles at most (1024 threads)
    const int tile = (n + 7) / 8 <= 7 ? (n + 7) / 8 : (n + 31) / 32;
    const size_t lds_sw = tile <= 7 ? patch_sweep_lds_bytes(tp.d, cond, p, t, tp.max_faces, tile) : 0;
    if (tile <= 7 && lds_sw <= kMaxLdsBytes - 1024 && threads == 0) {
      const int nt = (n + tile - 1) / tile;
      const int th = std::max(64, (nt * nt + 63) / 64 * 64);
      static bool attr[8] = {false, false, false, false, false, false, false, false};
#define HHO_SWEEP(TL)                                                                                            \
  case TL:                                                                                                       \
    if (!attr[TL]) {                                                                                             \
      if (hipFuncSetAttribute((const void *)k_patch_sweep<TL>, hipFuncAttributeMaxDynamicSharedMemorySize,       \
                              (int)(kMaxLdsBytes - 1024)) != hipSuccess)                                         \
        fail(HHO_E_DEVICE, "patch setup: cannot reserve LDS");                                                   \
      attr[TL] = true;                                                                                           \
    }                                                                                                            \
    hipLaunchKernelGGL((k_patch_sweep<TL>), dim3(tp.nc), dim3(th), lds_sw, s, tp, cond, p, t, bsr, cpl, spp, sinv, \
                       xinv, sig, err);                                                                          \
    return;
      switch (tile) {
        HHO_SWEEP(1)
        HHO_SWEEP(2)
        HHO_SWEEP(3)
        HHO_SWEEP(4)
        HHO_SWEEP(5)
        HHO_SWEEP(6)
        HHO_SWEEP(7)
        default:
          break;
      }
#undef HHO_SWEEP
    }
  }
  // LDS-resident factorisation when the packed patch fits the 160 KB of a CDNA4 CU
  const size_t packed = patch_lds_packed_bytes(tp.d, cond, p, t, tp.max_faces);
  const size_t budget = kMaxLdsBytes - 1024;  // leaves room for the kernel's static LDS
  if (packed <= budget) {
    static bool attr_set = false;
    if (!attr_set) {
      if (hipFuncSetAttribute((const void *)k_patch_setup_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)budget) != hipSuccess)
        fail(HHO_E_DEVICE, "patch setup: cannot reserve 160 KB of LDS");
      attr_set = true;
    }
    // threads per cell from the patch size (the kernel adapts to any multiple of 64 up to 512)
    const int n = tp.max_faces * ((cond == 1) ? p : tp.d * p);
    if (threads <= 0) threads = n <= 16 ? 64 : n <= 48 ? 128 : n <= 96 ? 256 : kPatchThreads;
    hipLaunchKernelGGL(k_patch_setup_lds, dim3(tp.nc), dim3(threads), packed, s, tp, cond, p, t, bsr, cpl, spp, sinv,
                       xinv, sig, err);
    return;
  }
  hipLaunchKernelGGL(k_patch_setup, dim3(tp.nc), dim3(kBlock), lds, s, tp, cond, p, t, bsr, cpl, spp, sinv, xinv,
                     sig, scratch, err);
}
template <typename Tout, typename Tin>
void launch_convert(const Tin *in, Tout *out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Tout, Tin>), dim3(grid_for(n)), dim3(kBlock), 0, s, in, out, n);
}
template void launch_convert<float, double>(const double *, float *, int64_t, hipStream_t);
template void launch_convert<double, float>(const float *, double *, int64_t, hipStream_t);
template void launch_convert<bf16, double>(const double *, bf16 *, int64_t, hipStream_t);

void launch_densify(const DTopo &tp, const DLevel<double> &L, int border, double *D, int64_t ld, hipStream_t s) {
  const int bs = (L.cond == 1) ? L.p : tp.d * L.p;
  int64_t total = tp.nnzb * bs * bs + tp.ncf * tp.d * L.p * L.t +
                  ((L.cond == 1) ? (int64_t)tp.nc * L.t * L.t : 0) + (border ? tp.nc : 0);
  hipLaunchKernelGGL(k_densify, dim3(grid_for(total)), dim3(kBlock), 0, s, tp, L, border, D, ld);
}
void launch_eye_right(double *D, int64_t n, int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(k_eye_right, dim3(grid_for(n)), dim3(kBlock), 0, s, D, n, ld);
}
void launch_gj_step(double *D, int64_t n, int64_t ld, int64_t k, double *colbuf, int *err, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kBlock), 0, s, D, n, ld, k, colbuf, err);
  hipLaunchKernelGGL(k_gj_elim, dim3(grid_for(n * 2 * n)), dim3(kBlock), 0, s, D, n, ld, k, colbuf);
}
void launch_dense_matvec(const double *Dinv, int64_t n, int64_t ld, int border, const double *x, double *y,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_dense_matvec, dim3(grid_for(n * kWave)), dim3(kBlock), 0, s, Dinv, n, ld, border, x, y);
}

}  // namespace hho
