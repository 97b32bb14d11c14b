// Arnoldi orthogonalisation of the (flexible) GMRES iterations of Section 3.3:
// classical Gram-Schmidt, once (coarse GMRES) or twice (outer FGMRES), with the
// Givens update of the Hessenberg column and the residual estimate done on the
// device by a one-block finishing kernel.
//
// Each thread owns E vector entries; for every entry it loads V_0..V_j (all
// loads independent), so the memory system sees (j+1) streams at full width.
// The j+1 per-thread dot products are summed over a wavefront by a butterfly
// that halves the number of live sums per exchange (NV-1 + 6-log2(NV) exchanges
// instead of 6 per sum), then over the block's waves through LDS, giving one
// partial per (vector, block); a one-block kernel adds the partials in a fixed
// order (deterministic).  The finishing work is a separate launch rather than
// the "last block to arrive" idiom: on a chip whose L2 caches are private to
// each die, the device-scope fence that idiom needs in every block writes back
// and invalidates that die's L2, which costs far more than a launch.
#include "dev_common.h"
#include "device.h"

namespace hho {
namespace {

constexpr int kOrthThreads = 512;
constexpr int kOrthMaxBlocks = 256;

// Block-level: partial[i * gridDim.x + blockIdx.x] = sum over the block of acc[i], i < nv.
template <int NV>
__device__ inline void block_multi_partial(double (&acc)[NV], int nv, double *partial) {
  __shared__ double red[kOrthThreads / kWave][NV];
  wave_multi_sum<NV>(acc);
  constexpr int shift = 6 - log2i<NV>();
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if ((lane & ((1 << shift) - 1)) == 0) red[wid][lane >> shift] = acc[0];
  __syncthreads();
  const int nwv = blockDim.x / kWave;  // waves of this launch (<= kOrthThreads / kWave)
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double s = 0;
    for (int w_ = 0; w_ < nwv; ++w_) s += red[w_][i];
    partial[(int64_t)i * gridDim.x + blockIdx.x] = s;
  }
}

// MODE 0: h1 = V^T w.
// MODE 1: w -= V h1, then h2 = V^T w.
// MODE 2: w -= V h (h = h2 if cgs2 else h1), then |w|^2 -> H column j, Givens, residual.
// MODE 3: h1 = V^T w and |w|^2 in one pass (classical Gram-Schmidt once, the new
//         norm by |w - V h1|^2 = |w|^2 - |h1|^2 for orthonormal V).
// MODE 4: V_{j+1} = (w - V h1) / h_{j+1,j} (the Hessenberg column already complete).
template <typename T, int NV, int MODE>
__global__ void __launch_bounds__(kOrthThreads) k_orth(int64_t n, int j, int E, const T *__restrict__ V,
                                                        int64_t ldv, T *__restrict__ w, double *partial,
                                                        GmresState *st, int cgs2) {
  if (st->done) return;
  __shared__ double h[NV];
  if (MODE != 0 && MODE != 3) {
    const double *src = (MODE == 2 && cgs2) ? st->h2 : st->h1;
    for (int i = threadIdx.x; i < NV; i += blockDim.x) h[i] = (i <= j) ? src[i] : 0.0;
    __syncthreads();
  }
  const double inv = (MODE == 4) ? st->inv_hnext : 1.0;
  const int nv = j + 1;
  double acc[NV], ww = 0;
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // vectors are taken eight at a time (eight independent loads in flight per
  // lane); the empty asm keeps the compiler from hoisting every load of the
  // entry ahead, which would cost registers and occupancy
#pragma unroll 1
  for (int e = 0; e < E && k < n; ++e, k += stride) {
    double wk = (double)w[k];
    const T *Vk = V + k;
    if (MODE != 0 && MODE != 3) {
#pragma unroll
      for (int c = 0; c < NV / 8; ++c) {
        if (c * 8 < nv) {
          double v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = (double)Vk[(int64_t)min(c * 8 + q, nv - 1) * ldv];
#pragma unroll
          for (int q = 0; q < 8; ++q) wk -= h[c * 8 + q] * v[q];  // h = 0 past column j
        }
        asm volatile("" ::: "memory");
      }
      if (MODE == 4) {
        const_cast<T *>(V)[(int64_t)nv * ldv + k] = (T)(wk * inv);
        continue;
      }
      w[k] = (T)wk;
      wk = (double)(T)wk;
    }
    if (MODE == 3) ww += wk * wk;
    if (MODE == 2) {
      acc[0] += wk * wk;
    } else {
#pragma unroll
      for (int c = 0; c < NV / 8; ++c) {
        if (c * 8 < nv) {
          double v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = (double)Vk[(int64_t)min(c * 8 + q, nv - 1) * ldv];
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[c * 8 + q] += v[q] * wk;  // sums past column j are unused
        }
        asm volatile("" ::: "memory");
      }
    }
  }
  if (MODE == 4) return;
  if (MODE == 2) {
    __shared__ double red[16];
    const double s = block_sum(acc[0], red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  } else if (MODE == 3) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i == nv) acc[i] = ww;  // the slot after the dots (its dot sum is unused)
    block_multi_partial<NV>(acc, nv + 1, partial);
  } else {
    block_multi_partial<NV>(acc, nv, partial);
  }
}

// The sums of MODE 3 split over blocks: blockIdx.y takes the eight sums
// 8 y .. 8 y + 7 of V_i^T w (i <= j) and w^T w (i = j + 1), so that a lane keeps
// all of its loads in flight at once (more blocks, one short chain each) rather
// than walking every basis vector; partial[i * gridDim.x + blockIdx.x] as MODE 3.
template <typename T>
__global__ void __launch_bounds__(kOrthThreads) k_orth_dots8(int64_t n, int j, int E, const T *__restrict__ V,
                                                             int64_t ldv, const T *__restrict__ w, double *partial,
                                                             const GmresState *st) {
  if (st->done) return;
  const int nv = j + 1;  // dot products; sum nv is |w|^2
  const int i0 = blockIdx.y * 8;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int e = 0; e < E && k < n; ++e, k += stride) {
    const double wk = (double)w[k];
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q;
      v[q] = (i < nv) ? (double)V[(int64_t)i * ldv + k] : wk;  // past sum nv: unused
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] += v[q] * wk;
  }
  block_multi_partial<8>(acc, min(8, nv + 1 - i0), partial + (int64_t)i0 * gridDim.x);
}

// Completes column j of the Hessenberg matrix (h1 (+ h2) above the diagonal,
// sqrt(nn) below), applies the previous Givens rotations and the new one, and
// updates the residual estimate and the convergence flag.  Whole block; the
// column and rotations are staged in LDS and one thread runs the dependent chain.
__device__ void givens_column(GmresState *st, int j, int cgs2, double nn) {
  __shared__ double col[kMaxRestartH + 1], cs[kMaxRestartH], sn[kMaxRestartH];
  for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = cgs2 ? st->h1[i] + st->h2[i] : st->h1[i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    cs[i] = st->cs[i];
    sn[i] = st->sn[i];
  }
  __syncthreads();
  const double hn = sqrt(nn);
  if (threadIdx.x == 0) {
    // previous rotations; the running entry is carried in a register so that the
    // loads of col, cs, sn do not wait on the stores
    double a = col[0];
    for (int i = 0; i < j; ++i) {
      const double b = col[i + 1];
      col[i] = cs[i] * a + sn[i] * b;
      a = -sn[i] * a + cs[i] * b;
    }
    col[j] = a;
    col[j + 1] = hn;
    const double b = hn;
    const double rr = sqrt(a * a + b * b);
    const double c = (rr > 0) ? a / rr : 1.0, s_ = (rr > 0) ? b / rr : 0.0;
    st->cs[j] = c;
    st->sn[j] = s_;
    col[j] = rr;
    col[j + 1] = 0;
    const double gj = st->g[j];
    st->g[j] = c * gj;
    st->g[j + 1] = -s_ * gj;
    st->res = fabs(st->g[j + 1]);
    st->j = j + 1;
    st->its += 1;
    st->inv_hnext = (hn > 0) ? 1.0 / hn : 0.0;
    if (!isfinite(nn) || !isfinite(st->res)) {
      st->nan = 1;
      st->done = 1;
    }
    if (st->res <= st->rtol * st->bnorm || hn <= 1e-14 * st->beta) st->done = 1;
  }
  __syncthreads();
  const int R = kMaxRestartH;
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) st->H[i * R + j] = col[i];
}

// One block: sums the partials of k_orth in a fixed order.  MODE 0/1 store h1/h2;
// MODE 2 completes column j of the Hessenberg matrix, applies the Givens
// rotations and updates the residual estimate and the convergence flag; MODE 3
// stores h1 and completes the column with |w|^2 - |h1|^2 as the new norm squared.
template <int MODE>
__global__ void __launch_bounds__(1024) k_orth_finish(int G, int j, const double *partial, GmresState *st,
                                                      int cgs2) {
  if (st->done) return;
  __shared__ double hs[kMaxRestartH + 1];
  const int nv = j + 1;
  if (MODE == 0 || MODE == 1) {
    reduce_partials(partial, G, nv, hs);
    double *dst = (MODE == 0) ? st->h1 : st->h2;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) dst[i] = hs[i];
    return;
  }
  if (MODE == 3) {
    reduce_partials(partial, G, nv + 1, hs);
    for (int i = threadIdx.x; i < nv; i += blockDim.x) st->h1[i] = hs[i];
    __shared__ double nn;
    if (threadIdx.x < kWave) {
      double hh = 0;
      for (int i = threadIdx.x; i < nv; i += kWave) hh += hs[i] * hs[i];
      hh = wave_sum(hh);
      if (threadIdx.x == 0) nn = fmax(hs[nv] - hh, 0.0);
    }
    __syncthreads();
    givens_column(st, j, 0, nn);
    return;
  }
  reduce_partials(partial, G, 1, hs);
  givens_column(st, j, cgs2, hs[0]);
}

void orth_shape(int64_t n, int *grid, int *E) {
  const int64_t per = kOrthThreads;
  int64_t e = (n + per * kOrthMaxBlocks - 1) / (per * kOrthMaxBlocks);
  if (e < 1) e = 1;
  int64_t g = (n + per * e - 1) / (per * e);
  if (g < 1) g = 1;
  *grid = (int)g;
  *E = (int)e;
}

template <typename T, int MODE>
void launch_mode(int64_t n, int j, const T *V, int64_t ldv, T *w, double *partial, GmresState *st, int cgs2,
                 hipStream_t s) {
  int grid, E;
  orth_shape(n, &grid, &E);
  const int nv = j + 1 + (MODE == 3 ? 1 : 0);  // sums per block (MODE 3: the dots and |w|^2)
#define HHO_ORTH(NVC)                                                                                             \
  hipLaunchKernelGGL((k_orth<T, NVC, MODE>), dim3(grid), dim3(kOrthThreads), 0, s, n, j, E, V, ldv, w, partial, \
                     st, cgs2)
  if (nv <= 8)
    HHO_ORTH(8);
  else if (nv <= 16)
    HHO_ORTH(16);
  else if (nv <= 32)
    HHO_ORTH(32);
  else
    HHO_ORTH(64);
#undef HHO_ORTH
  if (MODE != 4)
    hipLaunchKernelGGL((k_orth_finish<MODE>), dim3(1), dim3(1024), 0, s, grid, j, (const double *)partial, st,
                       cgs2);  // 16 waves: about two sums per wave
}

// ---------------------------------------------------------------- batched problems
// Chunk c covers kSegChunk consecutive virtual entries of segment ch[c].p; the
// partials of a segment's chunks are summed (in chunk order) by one block per
// segment.  Blocks of a converged segment return at once.
__device__ inline int64_t seg_index(const SegInfo &g, int64_t e) { return e < g.fl ? g.fo + e : g.co + (e - g.fl); }

constexpr int kSegThreads = 256;

// Sum over chunks [c0, c1) of partial[k * G + c] for k < K (waves per sum, lanes split chunks).
__device__ inline void reduce_range(const double *partial, int G, int c0, int c1, int K, double *out) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int k = wid; k < K; k += nw) {
    double s = 0;
    for (int b = c0 + lane; b < c1; b += kWave) s += partial[(int64_t)k * G + b];
    s = wave_sum(s);
    if (lane == 0) out[k] = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kSegThreads) k_seg_sumsq(const SegChunk *ch, const SegInfo *seg, const double *r,
                                                            double *partial) {
  __shared__ double red[16];
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  double acc = 0;
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const double v = r[seg_index(g, (int64_t)c.e0 + e)];
    acc += v * v;
  }
  const double sm = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = sm;
}

__global__ void __launch_bounds__(kBlock) k_seg_norm_finish(const int32_t *chunk_ptr, int G, const double *partial,
                                                             GmresState *st_all, int *sdone, int which) {
  const int p = blockIdx.x;
  GmresState *st = st_all + p;
  __shared__ double nsum[1];
  if (which == 0 && st->done && st->nan) return;
  if (which == 2 && st->done) {  // its correction is in x already: no columns in the next cycle
    if (threadIdx.x == 0) st->j = 0;
    return;
  }
  reduce_range(partial, G, chunk_ptr[p], chunk_ptr[p + 1], 1, nsum);
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
    sdone[p] = st->done;
  }
}

__global__ void __launch_bounds__(kSegThreads) k_seg_scale(const SegChunk *ch, const SegInfo *seg, const double *x,
                                                            const GmresState *st, double *y) {
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  // a converged member's next basis vector is zero: the V-cycle and the
  // operator, which act on the whole union, then carry only zeros in its slice,
  // and the slice cannot grow with a stale scale
  const bool done = st[c.p].done != 0;
  const double a = st[c.p].inv_hnext;
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t i = seg_index(g, (int64_t)c.e0 + e);
    y[i] = done ? 0.0 : a * x[i];
  }
}

// MODE 0: h1 = V^T w; 1: w -= V h1, h2 = V^T w; 2: w -= V h, |w|^2 (per segment, per chunk partials)
template <int NV, int MODE>
__global__ void __launch_bounds__(kSegThreads) k_seg_orth(const SegChunk *ch, const SegInfo *seg, int j,
                                                           const double *__restrict__ V, int64_t ldv,
                                                           double *__restrict__ w, double *partial,
                                                           const GmresState *st_all, int cgs2) {
  const SegChunk c = ch[blockIdx.x];
  const GmresState *st = st_all + c.p;
  const int nv = j + 1;
  if (st->done) {  // converged segment: keep the partial layout defined
    if (threadIdx.x < (MODE == 2 ? 1 : nv)) partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const SegInfo g = seg[c.p];
  __shared__ double h[NV];
  if (MODE != 0) {
    const double *src = (MODE == 2 && cgs2) ? st->h2 : st->h1;
    for (int i = threadIdx.x; i < NV; i += blockDim.x) h[i] = (i <= j) ? src[i] : 0.0;
    __syncthreads();
  }
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0;
#pragma unroll 1
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t k = seg_index(g, (int64_t)c.e0 + e);
    double wk = w[k];
    const double *Vk = V + k;
    if (MODE != 0) {
#pragma unroll
      for (int cc = 0; cc < NV / 8; ++cc) {
        if (cc * 8 < nv) {
          double v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = Vk[(int64_t)min(cc * 8 + q, nv - 1) * ldv];
#pragma unroll
          for (int q = 0; q < 8; ++q) wk -= h[cc * 8 + q] * v[q];
        }
        asm volatile("" ::: "memory");
      }
      w[k] = wk;
    }
    if (MODE == 2) {
      acc[0] += wk * wk;
    } else {
#pragma unroll
      for (int cc = 0; cc < NV / 8; ++cc) {
        if (cc * 8 < nv) {
          double v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = Vk[(int64_t)min(cc * 8 + q, nv - 1) * ldv];
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[cc * 8 + q] += v[q] * wk;
        }
        asm volatile("" ::: "memory");
      }
    }
  }
  if (MODE == 2) {
    __shared__ double red[16];
    const double sm = block_sum(acc[0], red);
    if (threadIdx.x == 0) partial[blockIdx.x] = sm;
  } else {
    block_multi_partial<NV>(acc, nv, partial);
  }
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_seg_orth_finish(const int32_t *chunk_ptr, int G, int j,
                                                             const double *partial, GmresState *st_all, int *sdone,
                                                             int cgs2) {
  const int p = blockIdx.x;
  GmresState *st = st_all + p;
  if (st->done) return;
  __shared__ double hs[kMaxRestartH + 1];
  const int nv = j + 1;
  if (MODE != 2) {
    reduce_range(partial, G, chunk_ptr[p], chunk_ptr[p + 1], nv, hs);
    double *dst = (MODE == 0) ? st->h1 : st->h2;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) dst[i] = hs[i];
    return;
  }
  reduce_range(partial, G, chunk_ptr[p], chunk_ptr[p + 1], 1, hs);
  givens_column(st, j, cgs2, hs[0]);
  if (threadIdx.x == 0) sdone[p] = st->done;
}

// y = H^{-1} g per segment (one thread each)
__global__ void k_seg_solve_ls(int np, GmresState *st_all) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  GmresState *st = st_all + p;
  const int R = kMaxRestartH;
  const int jn = st->j;
  for (int i = jn - 1; i >= 0; --i) {
    double v = st->g[i];
    for (int k = i + 1; k < jn; ++k) v -= st->H[i * R + k] * st->y[k];
    const double hii = st->H[i * R + i];
    st->y[i] = (hii != 0) ? v / hii : 0.0;
  }
}

__global__ void __launch_bounds__(kSegThreads) k_seg_combine(const SegChunk *ch, const SegInfo *seg, const double *Z,
                                                              int64_t ldz, const GmresState *st_all, double *x) {
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  const GmresState *st = st_all + c.p;
  const int jn = st->j;
  __shared__ double y[kMaxRestartH];
  for (int i = threadIdx.x; i < jn; i += blockDim.x) y[i] = st->y[i];
  __syncthreads();
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t k = seg_index(g, (int64_t)c.e0 + e);
    double v = x[k];
    for (int i = 0; i < jn; ++i) v += y[i] * Z[i * ldz + k];
    x[k] = v;
  }
}

__global__ void __launch_bounds__(kSegThreads) k_seg_dot2(const SegChunk *ch, const SegInfo *seg, const double *z,
                                                           const double *v, double *partial) {
  __shared__ double red[16];
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  double a = 0, b = 0;
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t k = seg_index(g, (int64_t)c.e0 + e);
    a += v[k] * z[k];
    b += z[k] * z[k];
  }
  const double sa = block_sum(a, red);
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = sa;
    partial[(int64_t)gridDim.x + blockIdx.x] = sb;
  }
}

__global__ void __launch_bounds__(kBlock) k_seg_ratio(const int32_t *chunk_ptr, int G, const double *partial,
                                                       double *ratio) {
  const int p = blockIdx.x;
  __shared__ double s2[2];
  reduce_range(partial, G, chunk_ptr[p], chunk_ptr[p + 1], 2, s2);
  if (threadIdx.x == 0) ratio[p] = s2[1] > 0 ? s2[0] / s2[1] : 0.0;
}

__global__ void __launch_bounds__(kSegThreads) k_seg_axpy(const SegChunk *ch, const SegInfo *seg, const double *ratio,
                                                           const double *z, double *v) {
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  const double a = ratio[c.p];
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t k = seg_index(g, (int64_t)c.e0 + e);
    v[k] -= a * z[k];
  }
}

// ---- smoothing step of every segment on its own (batched problems)
// Per chunk: the Gram sums of the step's directions, NS = 5 for two directions
// (w2 may be null: one direction), NS = 9 for three (layouts of mr2_solve and
// mr3_solve).
template <typename T, int NS>
__global__ void __launch_bounds__(kSegThreads) k_seg_mr_dots(const SegChunk *ch, const SegInfo *seg, const T *w1,
                                                              const T *w2, const T *w3, const T *r,
                                                              double *partial) {
  __shared__ double red[16];
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  double v[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = 0;
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t i = seg_index(g, (int64_t)c.e0 + e);
    const double x1 = w1[i], x2 = w2 ? (double)w2[i] : 0.0, rr = r[i];
    if constexpr (NS == 5) {
      v[0] += x1 * x1;
      v[1] += x1 * x2;
      v[2] += x2 * x2;
      v[3] += x1 * rr;
      v[4] += x2 * rr;
    } else {
      const double x3 = w3[i];
      v[0] += x1 * x1;
      v[1] += x1 * x2;
      v[2] += x1 * x3;
      v[3] += x2 * x2;
      v[4] += x2 * x3;
      v[5] += x3 * x3;
      v[6] += x1 * rr;
      v[7] += x2 * rr;
      v[8] += x3 * rr;
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double sm = block_sum(v[k], red);
    if (threadIdx.x == 0) partial[(int64_t)k * gridDim.x + blockIdx.x] = sm;
  }
}

// one block per segment: its coefficients y[3p .. 3p + 2]
template <int NS>
__global__ void __launch_bounds__(kBlock) k_seg_mr_finish(const int32_t *chunk_ptr, int G, int m,
                                                           const double *partial, double *y) {
  const int p = blockIdx.x;
  __shared__ double S[NS];
  reduce_range(partial, G, chunk_ptr[p], chunk_ptr[p + 1], NS, S);
  if (threadIdx.x == 0) {
    double yy[3] = {0, 0, 0};
    if constexpr (NS == 5)
      mr2_solve(S, m, yy);
    else
      mr3_solve(S, m, yy);
    y[3 * p] = yy[0];
    y[3 * p + 1] = yy[1];
    y[3 * p + 2] = yy[2];
  }
}

// x += Z y_p, r -= W y_p on every chunk, with its segment's coefficients (z2/w2
// null: one Schwarz direction; z3/w3 null: no third direction)
template <typename T>
__global__ void __launch_bounds__(kSegThreads) k_seg_mr_update(const SegChunk *ch, const SegInfo *seg,
                                                                const double *y, const T *z1, const T *z2,
                                                                const T *z3, const T *w1, const T *w2, const T *w3,
                                                                T *x, T *r) {
  const SegChunk c = ch[blockIdx.x];
  const SegInfo g = seg[c.p];
  const T y1 = (T)y[3 * c.p], y2 = (T)y[3 * c.p + 1], y3 = (T)y[3 * c.p + 2];
  for (int e = threadIdx.x; e < c.len; e += blockDim.x) {
    const int64_t i = seg_index(g, (int64_t)c.e0 + e);
    if (z3) {
      const T a2 = z2 ? z2[i] : (T)0, b2 = w2 ? w2[i] : (T)0;
      x[i] += y1 * z1[i] + y2 * a2 + y3 * z3[i];
      r[i] -= y1 * w1[i] + y2 * b2 + y3 * w3[i];
    } else if (z2) {
      x[i] += y1 * z1[i] + y2 * z2[i];
      r[i] -= y1 * w1[i] + y2 * w2[i];
    } else {
      x[i] += y1 * z1[i];
      r[i] -= y1 * w1[i];
    }
  }
}

// flag = 1 when every segment's done flag is set (one block)
__global__ void __launch_bounds__(kBlock) k_seg_all_done(int np, const int *sdone, int *flag) {
  __shared__ double red[16];
  double c = 0;
  for (int p = threadIdx.x; p < np; p += blockDim.x) c += sdone[p] ? 1.0 : 0.0;
  c = block_sum(c, red);
  if (threadIdx.x == 0) *flag = (c == (double)np) ? 1 : 0;
}

}  // namespace

static_assert(kMaxRestartH <= 64, "orthogonalisation kernels handle at most 64 basis vectors");

template <typename T>
void launch_arnoldi_dots(int64_t n, int j, const T *V, int64_t ldv, const T *w, double *partial, GmresState *st,
                         hipStream_t s) {
  launch_mode<T, 0>(n, j, V, ldv, const_cast<T *>(w), partial, st, 0, s);
}
template <typename T>
void launch_arnoldi_cgs1(int64_t n, int j, T *V, int64_t ldv, const T *w, double *partial, GmresState *st,
                         hipStream_t s) {
  int grid, E;
  orth_shape(n, &grid, &E);
  const int groups = (j + 2 + 7) / 8;  // j + 1 dot products and |w|^2
  hipLaunchKernelGGL((k_orth_dots8<T>), dim3(grid, groups), dim3(kOrthThreads), 0, s, n, j, E, (const T *)V, ldv, w,
                     partial, (const GmresState *)st);
  hipLaunchKernelGGL((k_orth_finish<3>), dim3(1), dim3(1024), 0, s, grid, j, (const double *)partial, st, 0);
  launch_mode<T, 4>(n, j, V, ldv, const_cast<T *>(w), partial, st, 0, s);
}
template <typename T>
void launch_arnoldi_update(int64_t n, int j, const T *V, int64_t ldv, T *w, double *partial, GmresState *st,
                           int pass, int cgs2, hipStream_t s) {
  if (pass == 1)
    launch_mode<T, 1>(n, j, V, ldv, w, partial, st, cgs2, s);
  else
    launch_mode<T, 2>(n, j, V, ldv, w, partial, st, cgs2, s);
}


void launch_seg_sumsq(int nchunks, const SegChunk *ch, const SegInfo *seg, const double *r, double *partial,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_seg_sumsq, dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, r, partial);
}
void launch_seg_norm_finish(int np, const int32_t *chunk_ptr, int nchunks, const double *partial, GmresState *st,
                            int *sdone, int which, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_norm_finish, dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, partial, st, sdone, which);
}
void launch_seg_scale(int nchunks, const SegChunk *ch, const SegInfo *seg, const double *x, const GmresState *st,
                      double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_scale, dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, x, st, y);
}
void launch_seg_arnoldi(int mode, int nchunks, const SegChunk *ch, const SegInfo *seg, int np,
                        const int32_t *chunk_ptr, int j, const double *V, int64_t ldv, double *w, double *partial,
                        GmresState *st, int *sdone, int cgs2, hipStream_t s) {
  const int nv = j + 1;
#define HHO_SEG(NVC, M)                                                                                          \
  hipLaunchKernelGGL((k_seg_orth<NVC, M>), dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, j, V, ldv, w, partial, \
                     (const GmresState *)st, cgs2)
#define HHO_SEG_NV(M)         \
  if (nv <= 8)                \
    HHO_SEG(8, M);            \
  else if (nv <= 16)          \
    HHO_SEG(16, M);           \
  else if (nv <= 32)          \
    HHO_SEG(32, M);           \
  else                        \
    HHO_SEG(64, M);
  if (mode == 0) {
    HHO_SEG_NV(0)
    hipLaunchKernelGGL((k_seg_orth_finish<0>), dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, j,
                       (const double *)partial, st, sdone, cgs2);
  } else if (mode == 1) {
    HHO_SEG_NV(1)
    hipLaunchKernelGGL((k_seg_orth_finish<1>), dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, j,
                       (const double *)partial, st, sdone, cgs2);
  } else {
    HHO_SEG_NV(2)
    hipLaunchKernelGGL((k_seg_orth_finish<2>), dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, j,
                       (const double *)partial, st, sdone, cgs2);
  }
#undef HHO_SEG_NV
#undef HHO_SEG
}
void launch_seg_solve_ls(int np, GmresState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_solve_ls, dim3((np + 63) / 64), dim3(64), 0, s, np, st);
}
void launch_seg_combine(int nchunks, const SegChunk *ch, const SegInfo *seg, const double *Z, int64_t ldz,
                        const GmresState *st, double *x, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_combine, dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, Z, ldz, st, x);
}
void launch_seg_project(int np, const int32_t *chunk_ptr, int nchunks, const SegChunk *ch, const SegInfo *seg,
                        const double *z, double *v, double *partial, double *ratio, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_dot2, dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, z, (const double *)v, partial);
  hipLaunchKernelGGL(k_seg_ratio, dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, (const double *)partial, ratio);
  hipLaunchKernelGGL(k_seg_axpy, dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, (const double *)ratio, z, v);
}

template <typename T>
void launch_seg_mr(int nchunks, const SegChunk *ch, const SegInfo *seg, int np, const int32_t *chunk_ptr, int m,
                   const T *z1, const T *z2, const T *z3, const T *w1, const T *w2, const T *w3, T *x, T *r,
                   double *partial, double *y, hipStream_t s) {
  if (m != 2) z2 = w2 = nullptr;
  if (z3) {
    hipLaunchKernelGGL((k_seg_mr_dots<T, 9>), dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, w1, w2, w3, r, partial);
    hipLaunchKernelGGL((k_seg_mr_finish<9>), dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, m,
                       (const double *)partial, y);
  } else {
    hipLaunchKernelGGL((k_seg_mr_dots<T, 5>), dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, w1, w2,
                       (const T *)nullptr, r, partial);
    hipLaunchKernelGGL((k_seg_mr_finish<5>), dim3(np), dim3(kBlock), 0, s, chunk_ptr, nchunks, m,
                       (const double *)partial, y);
  }
  hipLaunchKernelGGL((k_seg_mr_update<T>), dim3(nchunks), dim3(kSegThreads), 0, s, ch, seg, (const double *)y, z1, z2,
                     z3, w1, w2, w3, x, r);
}
void launch_seg_all_done(int np, const int *sdone, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_all_done, dim3(1), dim3(kBlock), 0, s, np, sdone, flag);
}

#define HHO_INST(T)                                                                                              \
  template void launch_arnoldi_dots<T>(int64_t, int, const T *, int64_t, const T *, double *, GmresState *,     \
                                       hipStream_t);                                                           \
  template void launch_arnoldi_update<T>(int64_t, int, const T *, int64_t, T *, double *, GmresState *, int,    \
                                         int, hipStream_t);                                                      \
  template void launch_arnoldi_cgs1<T>(int64_t, int, T *, int64_t, const T *, double *, GmresState *, hipStream_t); \
  template void launch_seg_mr<T>(int, const SegChunk *, const SegInfo *, int, const int32_t *, int, const T *,     \
                                 const T *, const T *, const T *, const T *, const T *, T *, T *, double *, double *, \
                                 hipStream_t);
HHO_INST(double)
HHO_INST(float)
#undef HHO_INST

}  // namespace hho
