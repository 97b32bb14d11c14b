// Zero-fill incomplete LU of a level operator, the preconditioner of the
// paper's smoother (Section 3.3: a few GMRES iterations preconditioned by ILU;
// Section 5.2 fixes two), in the natural ordering of the level's unknowns
// (faces, then cells) on the structural pattern of the condensed operator
// (every cell's dense block over its unknowns, zeros included).
//
// Exact, not iterative: the factorisation eliminates row by row in the natural
// order (for each k < i of row i in increasing order, l_ik = a_ik / u_kk, then
// row k's part right of its diagonal is subtracted where row i's pattern has
// it), the triangular solves substitute row by row; both run one dependency
// level at a time (a level = rows whose earlier neighbours are all in earlier
// levels), one wave per row.  Rows of one face (or one cell) share a column
// list.
#include <cstdint>
#include <mutex>

#include "dev_common.h"
#include "device.h"
#include "internal.h"

namespace hho {
namespace {

constexpr int kIluWaves = 4;  // rows per block

__device__ inline int64_t ilu_group(const IluDev &I, int64_t i) {
  const int dp = I.d * I.p;
  return i < I.nface ? i / dp : I.nface / dp + (i - I.nface) / I.t;
}

// first position in cols[0, n) not below v
__device__ inline int lower_bound_i32(const int32_t *cols, int n, int32_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cols[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// block index of (f, g) in the face-block rows (columns sorted per row), or -1
__device__ inline int bsr_block(const DTopo &tp, int f, int g) {
  const int rb = tp.rowptr[f], n = tp.rowptr[f + 1] - rb;
  const int pos = lower_bound_i32(tp.col + rb, n, g);
  return (pos < n && tp.col[rb + pos] == g) ? rb + pos : -1;
}

// position of face f in cell T's face list
__device__ inline int face_in_cell(const DTopo &tp, int T, int f) {
  for (int e = tp.cptr[T]; e < tp.cptr[T + 1]; ++e)
    if (tp.cface[e] == f) return e;
  return -1;
}

// value of the level operator at (i, j) (a position of the pattern)
__device__ double op_entry(const DTopo &tp, const DLevel<double> &L, int64_t i, int64_t j) {
  const int d = tp.d, p = L.p, t = L.t, dp = d * p;
  const bool fi = i < L.nface, fj = j < L.nface;
  if (fi && fj) {
    const int f = (int)(i / dp), g = (int)(j / dp), ri = (int)(i % dp), rj = (int)(j % dp);
    const int b = bsr_block(tp, f, g);
    if (b < 0) return 0.0;
    if (L.cond == 1) {
      if (ri / p != rj / p) return 0.0;  // s (x) I_d: no coupling between components
      return L.bsr[((int64_t)b * p + ri % p) * p + rj % p];
    }
    return L.bsr[((int64_t)b * dp + ri) * dp + rj];
  }
  if (fi != fj) {  // face row and cell column or the reverse (the operator is symmetric)
    const int64_t fr = fi ? i : j, cr = fi ? j : i;
    const int f = (int)(fr / dp), cf = (int)(fr % dp);
    const int T = (int)((cr - L.nface) / t), q = (int)((cr - L.nface) % t);
    const int e = face_in_cell(tp, T, f);
    if (e < 0) return 0.0;
    if (L.cond == 1) return L.cpl[((int64_t)e * dp + cf) * t + q];
    return L.cpl[(int64_t)e * dp + cf];
  }
  const int T = (int)((i - L.nface) / t), q = (int)((i - L.nface) % t);
  const int T2 = (int)((j - L.nface) / t), q2 = (int)((j - L.nface) % t);
  if (T != T2 || L.cond != 1) return 0.0;
  return L.spp[((int64_t)T * t + q) * t + q2];
}

__global__ void __launch_bounds__(kIluWaves * kWave) k_ilu_fill(DTopo tp, DLevel<double> L, IluDev I) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = (int64_t)blockIdx.x * kIluWaves + threadIdx.x / kWave;
  if (i >= I.N) return;
  const int64_t g = ilu_group(I, i);
  const int64_t c0 = I.gptr[g];
  const int n = (int)(I.gptr[g + 1] - c0);
  double *v = I.LU + I.voff[i];
  for (int e = lane; e < n; e += kWave) v[e] = op_entry(tp, L, i, I.gcol[c0 + e]);
}

// rows[0, n) of one dependency level; row values staged in LDS (maxrow per wave)
__global__ void __launch_bounds__(kIluWaves * kWave) k_ilu_factor(IluDev I, const int32_t *rows, int n, int maxrow,
                                                                   int *err) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int r = blockIdx.x * kIluWaves + w;
  if (r >= n) return;
  const int64_t i = rows[r];
  const int64_t g = ilu_group(I, i);
  const int64_t c0 = I.gptr[g];
  const int len = (int)(I.gptr[g + 1] - c0);
  const int32_t *cols = I.gcol + c0;
  double *rb = lds + (int64_t)w * maxrow;
  double *vi = I.LU + I.voff[i];
  for (int e = lane; e < len; e += kWave) rb[e] = vi[e];
  wave_fence();
  for (int idx = 0; idx < len; ++idx) {
    const int64_t k = cols[idx];
    if (k >= i) break;
    const double ukk = I.LU[I.diag[k]];
    if (ukk == 0.0) {
      if (lane == 0) err[0] = (int)i + 1;
      continue;
    }
    const double lik = rb[idx] / ukk;
    wave_fence();
    if (lane == 0) rb[idx] = lik;
    const int64_t gk = ilu_group(I, k);
    const int64_t ck0 = I.gptr[gk];
    const int lenk = (int)(I.gptr[gk + 1] - ck0);
    const int dk = (int)(I.diag[k] - I.voff[k]);
    const double *vk = I.LU + I.voff[k];
    for (int tpos = dk + 1 + lane; tpos < lenk; tpos += kWave) {
      const int32_t j = I.gcol[ck0 + tpos];
      const int pos = lower_bound_i32(cols, len, j);
      if (pos < len && cols[pos] == j) rb[pos] -= lik * vk[tpos];
    }
    wave_fence();
  }
  for (int e = lane; e < len; e += kWave) vi[e] = rb[e];
  const int di = (int)(I.diag[i] - I.voff[i]);
  if (lane == 0 && rb[di] == 0.0) err[0] = (int)i + 1;
}

// y_i = b_i - sum_{k < i} l_ik y_k for the rows of one level (L unit lower)
__global__ void __launch_bounds__(kIluWaves * kWave) k_ilu_lsolve(IluDev I, const int32_t *rows, int n,
                                                                   const double *b, double *y) {
  const int lane = threadIdx.x % kWave;
  const int r = blockIdx.x * kIluWaves + threadIdx.x / kWave;
  if (r >= n) return;
  const int64_t i = rows[r];
  const int64_t g = ilu_group(I, i);
  const int64_t c0 = I.gptr[g];
  const int dl = (int)(I.diag[i] - I.voff[i]);
  const double *vi = I.LU + I.voff[i];
  double s = 0;
  for (int e = lane; e < dl; e += kWave) s += vi[e] * y[I.gcol[c0 + e]];
  s = wave_sum(s);
  if (lane == 0) y[i] = b[i] - s;
}

// x_i = (x_i - sum_{j > i} u_ij x_j) / u_ii for the rows of one level, in place
__global__ void __launch_bounds__(kIluWaves * kWave) k_ilu_usolve(IluDev I, const int32_t *rows, int n, double *x) {
  const int lane = threadIdx.x % kWave;
  const int r = blockIdx.x * kIluWaves + threadIdx.x / kWave;
  if (r >= n) return;
  const int64_t i = rows[r];
  const int64_t g = ilu_group(I, i);
  const int64_t c0 = I.gptr[g];
  const int len = (int)(I.gptr[g + 1] - c0);
  const int dl = (int)(I.diag[i] - I.voff[i]);
  const double *vi = I.LU + I.voff[i];
  double s = 0;
  for (int e = dl + 1 + lane; e < len; e += kWave) s += vi[e] * x[I.gcol[c0 + e]];
  s = wave_sum(s);
  if (lane == 0) x[i] = (x[i] - s) / vi[dl];
}

inline unsigned ilu_blocks(int64_t rows) { return (unsigned)((rows + kIluWaves - 1) / kIluWaves); }

}  // namespace

void launch_ilu_fill(const DTopo &tp, const DLevel<double> &L, const IluDev &I, hipStream_t s) {
  if (I.N > 0) hipLaunchKernelGGL(k_ilu_fill, dim3(ilu_blocks(I.N)), dim3(kIluWaves * kWave), 0, s, tp, L, I);
}

void launch_ilu_factor(const IluDev &I, const int32_t *lrows, const int32_t *lptr, int nlev, int maxrow, int *err,
                       hipStream_t s) {
  const size_t lds = (size_t)kIluWaves * maxrow * sizeof(double);
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    attr = hipFuncSetAttribute((const void *)k_ilu_factor, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMaxLdsBytes - 1024));
  });
  if (attr != hipSuccess) fail(HHO_E_DEVICE, "ILU factorisation: cannot reserve LDS");
  for (int lv = 0; lv < nlev; ++lv) {
    const int n = lptr[lv + 1] - lptr[lv];
    hipLaunchKernelGGL(k_ilu_factor, dim3(ilu_blocks(n)), dim3(kIluWaves * kWave), lds, s, I, lrows + lptr[lv], n,
                       maxrow, err);
  }
}

void launch_ilu_apply(const IluDev &I, const int32_t *lrows, const int32_t *lptr, int nlevL, const int32_t *urows,
                      const int32_t *uptr, int nlevU, const double *r, double *z, hipStream_t s) {
  for (int lv = 0; lv < nlevL; ++lv) {
    const int n = lptr[lv + 1] - lptr[lv];
    hipLaunchKernelGGL(k_ilu_lsolve, dim3(ilu_blocks(n)), dim3(kIluWaves * kWave), 0, s, I, lrows + lptr[lv], n, r, z);
  }
  for (int lv = 0; lv < nlevU; ++lv) {
    const int n = uptr[lv + 1] - uptr[lv];
    hipLaunchKernelGGL(k_ilu_usolve, dim3(ilu_blocks(n)), dim3(kIluWaves * kWave), 0, s, I, urows + uptr[lv], n, z);
  }
}

}  // namespace hho
