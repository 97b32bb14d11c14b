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

// One butterfly exchange across lanes (lane ^ O): the lower lane keeps the first
// H sums and the upper lane the second H, each adding its partner's copy.
template <int NV, int H, int O>
__device__ inline void halve(double (&acc)[NV], bool upper) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = upper ? acc[i] : acc[i + H];
    const double keep = upper ? acc[i + H] : acc[i];
    acc[i] = keep + __shfl_xor(send, O, kWave);
  }
}

template <int NV, int LIVE, int O>
__device__ inline void multi_sum_step(double (&acc)[NV], int lane) {
  if constexpr (O >= 1) {
    if constexpr (LIVE > 1) {
      halve<NV, LIVE / 2, O>(acc, (lane & O) != 0);
      multi_sum_step<NV, LIVE / 2, O / 2>(acc, lane);
    } else {
      acc[0] += __shfl_xor(acc[0], O, kWave);
      multi_sum_step<NV, 1, O / 2>(acc, lane);
    }
  }
}

// Sum over the 64 lanes of a wave of acc[0..NV) (NV a power of two <= 64).
// On return acc[0] holds, in every lane, the total of vector (lane >> (6 - log2 NV)).
template <int NV>
__device__ inline void wave_multi_sum(double (&acc)[NV]) {
  multi_sum_step<NV, NV, kWave / 2>(acc, threadIdx.x % kWave);
}

template <int NV>
constexpr int log2i() {
  return NV <= 1 ? 0 : 1 + log2i<NV / 2>();
}

// Block-level: partial[i * gridDim.x + blockIdx.x] = sum over the block of acc[i], i < nv.
template <int NV>
__device__ inline void block_multi_partial(double (&acc)[NV], int nv, double *partial) {
  __shared__ double red[kOrthThreads / kWave][NV];
  wave_multi_sum<NV>(acc);
  constexpr int shift = 6 - log2i<NV>();
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if ((lane & ((1 << shift) - 1)) == 0) red[wid][lane >> shift] = acc[0];
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    double s = 0;
#pragma unroll
    for (int w_ = 0; w_ < kOrthThreads / kWave; ++w_) s += red[w_][i];
    partial[(int64_t)i * gridDim.x + blockIdx.x] = s;
  }
}

// MODE 0: h1 = V^T w.
// MODE 1: w -= V h1, then h2 = V^T w.
// MODE 2: w -= V h (h = h2 if cgs2 else h1), then |w|^2 -> H column j, Givens, residual.
template <typename T, int NV, int MODE>
__global__ void __launch_bounds__(kOrthThreads) k_orth(int64_t n, int j, int E, const T *__restrict__ V,
                                                        int64_t ldv, T *__restrict__ w, double *partial,
                                                        GmresState *st, int cgs2) {
  if (st->done) return;
  __shared__ double h[NV];
  if (MODE != 0) {
    const double *src = (MODE == 2 && cgs2) ? st->h2 : st->h1;
    for (int i = threadIdx.x; i < NV; i += blockDim.x) h[i] = (i <= j) ? src[i] : 0.0;
    __syncthreads();
  }
  const int nv = j + 1;
  double acc[NV];
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
    if (MODE != 0) {
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
      w[k] = (T)wk;
      wk = (double)(T)wk;
    }
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
  if (MODE == 2) {
    __shared__ double red[16];
    const double s = block_sum(acc[0], red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  } else {
    block_multi_partial<NV>(acc, nv, partial);
  }
}

// One block: sums the partials of k_orth in a fixed order.  MODE 0/1 store h1/h2;
// MODE 2 completes column j of the Hessenberg matrix, applies the Givens
// rotations and updates the residual estimate and the convergence flag.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_orth_finish(int G, int j, const double *partial, GmresState *st,
                                                        int cgs2) {
  if (st->done) return;
  __shared__ double hs[kMaxRestartH + 1];
  const int nv = j + 1;
  if (MODE != 2) {
    reduce_partials(partial, G, nv, hs);
    double *dst = (MODE == 0) ? st->h1 : st->h2;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) dst[i] = hs[i];
    return;
  }
  // column j of H in LDS, previous rotations staged in LDS, then one thread
  // applies them (a dependent chain, kept out of global memory)
  __shared__ double col[kMaxRestartH + 1], cs[kMaxRestartH], sn[kMaxRestartH];
  for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = cgs2 ? st->h1[i] + st->h2[i] : st->h1[i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    cs[i] = st->cs[i];
    sn[i] = st->sn[i];
  }
  reduce_partials(partial, G, 1, hs);  // ends with a barrier
  const double nn = hs[0];
  const double hn = sqrt(nn);
  if (threadIdx.x == 0) {
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = cs[i] * a + sn[i] * b;
      col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    col[j + 1] = hn;
    const double a = col[j], b = hn;
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
  const int nv = j + 1;
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
  hipLaunchKernelGGL((k_orth_finish<MODE>), dim3(1), dim3(kBlock), 0, s, grid, j, (const double *)partial, st, cgs2);
}

}  // namespace

static_assert(kMaxRestartH <= 64, "orthogonalisation kernels handle at most 64 basis vectors");

template <typename T>
void launch_arnoldi_dots(int64_t n, int j, const T *V, int64_t ldv, const T *w, double *partial, GmresState *st,
                         hipStream_t s) {
  launch_mode<T, 0>(n, j, V, ldv, const_cast<T *>(w), partial, st, 0, s);
}
template <typename T>
void launch_arnoldi_update(int64_t n, int j, const T *V, int64_t ldv, T *w, double *partial, GmresState *st,
                           int pass, int cgs2, hipStream_t s) {
  if (pass == 1)
    launch_mode<T, 1>(n, j, V, ldv, w, partial, st, cgs2, s);
  else
    launch_mode<T, 2>(n, j, V, ldv, w, partial, st, cgs2, s);
}

#define HHO_INST(T)                                                                                              \
  template void launch_arnoldi_dots<T>(int64_t, int, const T *, int64_t, const T *, double *, GmresState *,     \
                                       hipStream_t);                                                           \
  template void launch_arnoldi_update<T>(int64_t, int, const T *, int64_t, T *, double *, GmresState *, int,    \
                                         int, hipStream_t);
HHO_INST(double)
HHO_INST(float)
#undef HHO_INST

}  // namespace hho
