// Face-block operator application with the block sizes fixed at compile time
// (one instantiation per (dimension, level degree, condensation variant)).
//
// y = S x (MODE 0) or y = b - S x (MODE 1) for the condensed operator of
// Section 3.2 stored as face-block rows (plus the cell couplings):
//  * v-cond: S_{FF'} = s_{FF'} (x) I_d, so a thread owns the face row (F, r) for
//    every velocity component c and reads each scalar block entry once for all
//    d components; the cell rows (T, q) use the same coupling array read by
//    column (lanes q contiguous) and S_TT by column (it is symmetric);
//  * v&p-cond: a thread owns one row of the d*p face block.
// The operator is symmetric, so the entry (r, k) of the block (F, F') equals the
// entry (k, r) of its mirror block (F', F): reading the mirror by columns gives
// lanes r consecutive addresses (coalesced) where the block itself would be
// read with a row stride.
// With SPLIT the face part of x is the sum of the two slot vectors x and xs1
// (Schwarz output), and xsum (if not null) receives that sum.
#include "dev_common.h"
#include "device.h"
#include "probe.h"

namespace hho {
namespace {

template <typename T, bool SPLIT>
__device__ inline T xface(const T *__restrict__ x, const T *__restrict__ xs1, int64_t i) {
  if (SPLIT) return x[i] + xs1[i];
  return x[i];
}

template <typename T, typename Sto, typename StoP, int D, int P, int TT, bool SPLIT, int MODE>
__global__ void __launch_bounds__(kBlock) k_spmv_v(DTopo tp, DLevel<T, Sto, StoP> L, const T *__restrict__ x,
                                                    const T *__restrict__ xs1, T *__restrict__ xsum,
                                                    const T *__restrict__ b, T *__restrict__ y) {
  constexpr int DP = D * P;
  const int64_t nfr = (int64_t)tp.nf * P;
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o >= nfr + (int64_t)tp.nc * TT) return;
  if (o < nfr) {
    const int f = (int)(o / P), r = (int)(o % P);
    T acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0;
    const int rb = tp.rowptr[f], re = tp.rowptr[f + 1];
    // U blocks in flight per step (small blocks: the loop is latency-bound);
    // a 1 x 1 block is its own mirror
    constexpr int U = DP <= 8 ? 4 : DP <= 16 ? 2 : 1;
    for (int b0 = rb; b0 < re; b0 += U) {
      int64_t fc[U], mb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = b0 + u < re;
        fc[u] = in ? tp.col[b0 + u] : 0;
        mb[u] = in ? (P == 1 ? b0 + u : tp.mirror[b0 + u]) : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (mb[u] < 0) continue;
        const Sto *blk = L.bsr + mb[u] * (P * P) + r;
        T bv[P];
#pragma unroll
        for (int k = 0; k < P; ++k) bv[k] = blk[k * P];
        const int64_t xo = fc[u] * DP;
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int k = 0; k < P; ++k) acc[c] += bv[k] * xface<T, SPLIT>(x, xs1, xo + c * P + k);
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int Tc = tp.fcell[2 * f + s];
      if (Tc < 0) continue;
      const int64_t e = (int64_t)tp.cptr[Tc] + tp.floc[2 * f + s];
      const Sto *cp = L.cpl + (e * DP + r) * TT;
      const T *xp = x + L.nface + (int64_t)Tc * TT;
      T xv[TT];
#pragma unroll
      for (int q = 0; q < TT; ++q) xv[q] = xp[q];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int q = 0; q < TT; ++q) acc[c] += cp[c * P * TT + q] * xv[q];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const int64_t i = (int64_t)f * DP + c * P + r;
      y[i] = (MODE == 1) ? (T)(b[i] - acc[c]) : acc[c];
      if (SPLIT && xsum) xsum[i] = x[i] + xs1[i];
    }
  } else {
    const int64_t oc = o - nfr;
    const int Tc = (int)(oc / TT), q = (int)(oc % TT);
    T acc = 0;
    const int eb = tp.cptr[Tc], ee = tp.cptr[Tc + 1];
    for (int e = eb; e < ee; ++e) {
      const int64_t xo = (int64_t)tp.cface[e] * DP;
      const Sto *cp = L.cpl + (int64_t)e * DP * TT + q;
#pragma unroll
      for (int j = 0; j < DP; ++j) acc += cp[j * TT] * xface<T, SPLIT>(x, xs1, xo + j);
    }
    const Sto *sp = L.spp + (int64_t)Tc * TT * TT + q;
    const T *xp = x + L.nface + (int64_t)Tc * TT;
#pragma unroll
    for (int q2 = 0; q2 < TT; ++q2) acc += sp[q2 * TT] * xp[q2];
    const int64_t i = L.nface + oc;
    y[i] = (MODE == 1) ? (T)(b[i] - acc) : acc;
    if (SPLIT && xsum) xsum[i] = x[i];
  }
}

// Lowest degree (k = 0, v-cond: one face mode, one pressure mode per cell): the
// rows are short, so G lanes share a row (its blocks, its two cells, or its
// cell's faces) and combine by shuffles; otherwise as k_spmv_v.
template <typename T, typename Sto, typename StoP, int D, int G, bool SPLIT, int MODE>
__global__ void __launch_bounds__(kBlock) k_spmv_v0(DTopo tp, DLevel<T, Sto, StoP> L, const T *__restrict__ x,
                                                     const T *__restrict__ xs1, T *__restrict__ xsum,
                                                     const T *__restrict__ b, T *__restrict__ y) {
  if (L.skip && *L.skip) return;
  const int64_t o = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (o >= (int64_t)tp.nf + tp.nc) return;  // uniform over the group
  if (o < tp.nf) {
    const int f = (int)o;
    T acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0;
    for (int bi = tp.rowptr[f] + lane; bi < tp.rowptr[f + 1]; bi += G) {
      const T a = (T)L.bsr[bi];  // a 1 x 1 block is its own mirror
      const int64_t xo = (int64_t)tp.col[bi] * D;
#pragma unroll
      for (int c = 0; c < D; ++c) acc[c] += a * xface<T, SPLIT>(x, xs1, xo + c);
    }
    if (lane < 2) {
      const int Tc = tp.fcell[2 * f + lane];
      if (Tc >= 0) {
        const int64_t e = (int64_t)tp.cptr[Tc] + tp.floc[2 * f + lane];
        const T xc = x[L.nface + Tc];
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] += L.cpl[e * D + c] * xc;
      }
    }
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = group_sum<G>(acc[c]);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const int64_t i = (int64_t)f * D + c;
        y[i] = (MODE == 1) ? (T)(b[i] - acc[c]) : acc[c];
        if (SPLIT && xsum) xsum[i] = x[i] + xs1[i];
      }
    }
  } else {
    const int Tc = (int)(o - tp.nf);
    T acc = 0;
    for (int e = tp.cptr[Tc] + lane; e < tp.cptr[Tc + 1]; e += G) {
      const int64_t xo = (int64_t)tp.cface[e] * D;
#pragma unroll
      for (int j = 0; j < D; ++j) acc += L.cpl[(int64_t)e * D + j] * xface<T, SPLIT>(x, xs1, xo + j);
    }
    if (lane == 0) acc += L.spp[Tc] * x[L.nface + Tc];
    acc = group_sum<G>(acc);
    if (lane == 0) {
      const int64_t i = L.nface + Tc;
      y[i] = (MODE == 1) ? (T)(b[i] - acc) : acc;
      if (SPLIT && xsum) xsum[i] = x[i];
    }
  }
}

// Lowest degree, v&p-cond (d x d face blocks, one mean pressure per cell): G lanes
// share a face row block (its blocks, read whole by one lane, and its two cells)
// or a cell row (its faces), combined by shuffles.
template <typename T, typename Sto, typename StoP, int BS, int G, bool SPLIT, int MODE>
__global__ void __launch_bounds__(kBlock) k_spmv_vp0(DTopo tp, DLevel<T, Sto, StoP> L, const T *__restrict__ x,
                                                      const T *__restrict__ xs1, T *__restrict__ xsum,
                                                      const T *__restrict__ b, T *__restrict__ y) {
  if (L.skip && *L.skip) return;
  const int64_t o = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (o >= (int64_t)tp.nf + tp.nc) return;  // uniform over the group
  if (o < tp.nf) {
    const int f = (int)o;
    T acc[BS];
#pragma unroll
    for (int i = 0; i < BS; ++i) acc[i] = 0;
    for (int bi = tp.rowptr[f] + lane; bi < tp.rowptr[f + 1]; bi += G) {
      const Sto *blk = L.bsr + (int64_t)bi * (BS * BS);
      const int64_t xo = (int64_t)tp.col[bi] * BS;
      T xv[BS];
#pragma unroll
      for (int k = 0; k < BS; ++k) xv[k] = xface<T, SPLIT>(x, xs1, xo + k);
#pragma unroll
      for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int k = 0; k < BS; ++k) acc[i] += blk[i * BS + k] * xv[k];
    }
    if (lane < 2) {
      const int Tc = tp.fcell[2 * f + lane];
      if (Tc >= 0) {
        const int64_t e = (int64_t)tp.cptr[Tc] + tp.floc[2 * f + lane];
        const T xc = x[L.nface + Tc];
#pragma unroll
        for (int i = 0; i < BS; ++i) acc[i] += L.cpl[e * BS + i] * xc;
      }
    }
#pragma unroll
    for (int i = 0; i < BS; ++i) acc[i] = group_sum<G>(acc[i]);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < BS; ++i) {
        const int64_t r = (int64_t)f * BS + i;
        y[r] = (MODE == 1) ? (T)(b[r] - acc[i]) : acc[i];
        if (SPLIT && xsum) xsum[r] = x[r] + xs1[r];
      }
    }
  } else {
    const int Tc = (int)(o - tp.nf);
    T acc = 0;
    for (int e = tp.cptr[Tc] + lane; e < tp.cptr[Tc + 1]; e += G) {
      const int64_t xo = (int64_t)tp.cface[e] * BS;
#pragma unroll
      for (int k = 0; k < BS; ++k) acc += L.cpl[(int64_t)e * BS + k] * xface<T, SPLIT>(x, xs1, xo + k);
    }
    acc = group_sum<G>(acc);
    if (lane == 0) {
      const int64_t r = L.nface + Tc;
      y[r] = (MODE == 1) ? (T)(b[r] - acc) : acc;
      if (SPLIT && xsum) xsum[r] = x[r];
    }
  }
}

template <typename T, typename Sto, typename StoP, int BS, bool SPLIT, int MODE>
__global__ void __launch_bounds__(kBlock) k_spmv_vp(DTopo tp, DLevel<T, Sto, StoP> L, const T *__restrict__ x,
                                                     const T *__restrict__ xs1, T *__restrict__ xsum,
                                                     const T *__restrict__ b, T *__restrict__ y) {
  const int64_t nfr = (int64_t)tp.nf * BS;
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o >= nfr + tp.nc) return;
  if (o < nfr) {
    const int f = (int)(o / BS), i = (int)(o % BS);
    T acc = 0;
    const int rb = tp.rowptr[f], re = tp.rowptr[f + 1];
    for (int bi = rb; bi < re; ++bi) {
      const int64_t xo = (int64_t)tp.col[bi] * BS;
      const Sto *blk = L.bsr + (int64_t)tp.mirror[bi] * (BS * BS) + i;
#pragma unroll
      for (int k = 0; k < BS; ++k) acc += blk[k * BS] * xface<T, SPLIT>(x, xs1, xo + k);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int Tc = tp.fcell[2 * f + s];
      if (Tc < 0) continue;
      const int64_t e = (int64_t)tp.cptr[Tc] + tp.floc[2 * f + s];
      acc += L.cpl[e * BS + i] * x[L.nface + Tc];
    }
    y[o] = (MODE == 1) ? (T)(b[o] - acc) : acc;
    if (SPLIT && xsum) xsum[o] = x[o] + xs1[o];
  } else {
    const int Tc = (int)(o - nfr);
    T acc = 0;
    const int eb = tp.cptr[Tc], ee = tp.cptr[Tc + 1];
    for (int e = eb; e < ee; ++e) {
      const int64_t xo = (int64_t)tp.cface[e] * BS;
      const Sto *cp = L.cpl + (int64_t)e * BS;
#pragma unroll
      for (int k = 0; k < BS; ++k) acc += cp[k] * xface<T, SPLIT>(x, xs1, xo + k);
    }
    y[o] = (MODE == 1) ? (T)(b[o] - acc) : acc;
    if (SPLIT && xsum) xsum[o] = x[o];
  }
}

constexpr int dimP(int d, int k) { return d == 2 ? k + 1 : (k + 1) * (k + 2) / 2; }
constexpr int dimT(int d, int k) { return d == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6; }

template <typename T, typename Sto, typename StoP, bool SPLIT, int MODE, int D, int K>
bool try_launch(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *x, const T *xs1, T *xsum, const T *b, T *y,
                hipStream_t s) {
  constexpr int P = dimP(D, K), TT = dimT(D, K);
  if (tp.d != D || L.p != P) return false;
  if (L.cond == 1) {
    if (L.t != TT) return false;
    const int bs = L.block > 0 ? L.block : kBlock;
    if (K == 0) {
      constexpr int G = 4;
      const int64_t total = ((int64_t)tp.nf + tp.nc) * G;
      const int grid = (int)((total + bs - 1) / bs);
      HHO_LAUNCH((k_spmv_v0<T, Sto, StoP, D, G, SPLIT, MODE>), dim3(grid), dim3(bs), 0, s, tp, L, x, xs1, xsum, b, y);
      return true;
    }
    const int64_t total = (int64_t)tp.nf * P + (int64_t)tp.nc * TT;
    const int grid = (int)((total + bs - 1) / bs);
    HHO_LAUNCH((k_spmv_v<T, Sto, StoP, D, P, TT, SPLIT, MODE>), dim3(grid), dim3(bs), 0, s, tp, L, x, xs1, xsum, b, y);
  } else {
    const int bs = L.block > 0 ? L.block : kBlock;
    if (K == 0) {
      constexpr int G = 4;
      const int64_t total = ((int64_t)tp.nf + tp.nc) * G;
      const int grid = (int)((total + bs - 1) / bs);
      HHO_LAUNCH((k_spmv_vp0<T, Sto, StoP, D, G, SPLIT, MODE>), dim3(grid), dim3(bs), 0, s, tp, L, x, xs1, xsum, b, y);
      return true;
    }
    const int64_t total = (int64_t)tp.nf * D * P + tp.nc;
    const int grid = (int)((total + bs - 1) / bs);
    HHO_LAUNCH((k_spmv_vp<T, Sto, StoP, D * P, SPLIT, MODE>), dim3(grid), dim3(bs), 0, s, tp, L, x, xs1, xsum, b, y);
  }
  return true;
}

template <typename T, typename Sto, typename StoP, bool SPLIT, int MODE>
bool dispatch(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *x, const T *xs1, T *xsum, const T *b, T *y,
              hipStream_t s) {
  return try_launch<T, Sto, StoP, SPLIT, MODE, 2, 0>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 2, 1>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 2, 2>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 2, 3>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 2, 4>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 3, 0>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 3, 1>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 3, 2>(tp, L, x, xs1, xsum, b, y, s) ||
         try_launch<T, Sto, StoP, SPLIT, MODE, 3, 3>(tp, L, x, xs1, xsum, b, y, s);
}

}  // namespace

template <typename T, typename Sto, typename StoP>
bool launch_spmv_fixed(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *x, const T *xs1, T *xsum, const T *b, T *y,
                       hipStream_t s) {
  if (tp.nf == 0 && tp.nc == 0) return true;
  if (b) return dispatch<T, Sto, StoP, false, 1>(tp, L, x, nullptr, nullptr, b, y, s);
  if (xs1) return dispatch<T, Sto, StoP, true, 0>(tp, L, x, xs1, xsum, nullptr, y, s);
  return dispatch<T, Sto, StoP, false, 0>(tp, L, x, nullptr, nullptr, nullptr, y, s);
}

template bool launch_spmv_fixed<double, double, double>(const DTopo &, const DLevel<double> &, const double *,
                                                        const double *, double *, const double *, double *,
                                                        hipStream_t);
template bool launch_spmv_fixed<float, float, float>(const DTopo &, const DLevel<float> &, const float *,
                                                     const float *, float *, const float *, float *, hipStream_t);
template bool launch_spmv_fixed<float, bf16, float>(const DTopo &, const DLevel<float, bf16, float> &,
                                                    const float *, const float *, float *, const float *, float *,
                                                    hipStream_t);

}  // namespace hho
