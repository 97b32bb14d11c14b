// Device-side helpers shared by the HIP translation units (CDNA wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hho {

// bfloat16 storage of operator and smoother values (the 16 high bits of an IEEE
// binary32): read as float, arithmetic in float.  Rounding from float is to the
// nearest, ties to even (add 0x7fff plus the lowest kept bit, drop 16 bits; NaN
// stays a quiet NaN).
struct bf16 {
  uint16_t bits;
  __host__ __device__ operator float() const { return __builtin_bit_cast(float, (uint32_t)bits << 16); }
};
__host__ __device__ inline bf16 to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40u)};  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}
// value conversion to a storage type (double -> float -> bf16 for bf16)
template <typename To>
struct StoreAs {
  template <typename From>
  __host__ __device__ static To from(From v) { return (To)v; }
};
template <>
struct StoreAs<bf16> {
  template <typename From>
  __host__ __device__ static bf16 from(From v) { return to_bf16((float)v); }
};

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kMaxRestart = 64;

// Sum over a 64-lane wavefront.
__device__ inline double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}

// Sum over the G lanes of a row group (G a power of two dividing 64); result in
// the group's first lane.
template <int G, typename T>
__device__ inline T group_sum(T v) {
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_down(v, o, G);
  return v;
}

// One butterfly exchange across lanes (lane ^ O): the lower lane keeps the first
// H sums and the upper lane the second H, each adding its partner's copy.
template <int NV, int H, int O, typename T>
__device__ inline void halve(T (&acc)[NV], bool upper) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const T send = upper ? acc[i] : acc[i + H];
    const T keep = upper ? acc[i + H] : acc[i];
    acc[i] = keep + __shfl_xor(send, O, kWave);
  }
}

template <int NV, int LIVE, int O, typename T>
__device__ inline void multi_sum_step(T (&acc)[NV], int lane) {
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

// Sum over the 64 lanes of a wave of acc[0..NV) (NV a power of two <= 64) in
// NV - 1 + 6 - log2(NV) exchanges (a butterfly that halves the live sums per
// exchange).  On return acc[0] holds, in every lane, the total of vector
// (lane >> (6 - log2 NV)).
template <int NV, typename T>
__device__ inline void wave_multi_sum(T (&acc)[NV]) {
  multi_sum_step<NV, NV, kWave / 2>(acc, threadIdx.x % kWave);
}

template <int NV>
constexpr int log2i() {
  return NV <= 1 ? 0 : 1 + log2i<NV / 2>();
}

// Block-wide sum (blockDim.x a multiple of 64, <= 1024); result valid in thread 0.
__device__ inline double block_sum(double v, double *lds /* >= 16 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    for (int i = 0; i < nw; ++i) r += lds[i];
  }
  __syncthreads();
  return r;
}

// Inside a one-block finishing kernel: out[k] = sum_b partial[k*G + b] for k < K.  Waves take
// the sums in turn, lanes split the G partials (parallel loads), the per-lane
// order and the wave tree are fixed, so the result is deterministic.  `out` must
// be visible to the whole block (LDS); a barrier ends the function.
__device__ inline void reduce_partials(const double *partial, int G, int K, double *out) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int k = wid; k < K; k += nw) {
    double s = 0;
    for (int b = lane; b < G; b += kWave) s += partial[(int64_t)k * G + b];
    s = wave_sum(s);
    if (lane == 0) out[k] = s;
  }
  __syncthreads();
}

// Coefficients of the smoothing step's minimal-residual update (Section 3.3: the
// GMRES(2) iterate started from zero is the minimal-residual combination of the
// first two preconditioned directions).  S holds the Gram sums of the operator
// images w_i and their products with the residual:
//   two directions  S = {w1.w1, w1.w2, w2.w2, w1.r, w2.r}            (m = 1: w1 only)
//   three           S = {a11, a12, a13, a22, a23, a33, g1, g2, g3}   (m = 1: w2 dropped)
// A direction that is numerically dependent on the earlier ones gets a zero
// coefficient; non-finite results give zero coefficients.
__device__ inline void mr2_solve(const double *S, int m, double *y) {
  double y1 = 0, y2 = 0;
  const double det = S[0] * S[2] - S[1] * S[1];
  if (m == 2 && det > 1e-14 * S[0] * S[2]) {
    y1 = (S[2] * S[3] - S[1] * S[4]) / det;
    y2 = (S[0] * S[4] - S[1] * S[3]) / det;
  } else if (S[0] > 0) {
    y1 = S[3] / S[0];
  }
  if (!isfinite(y1) || !isfinite(y2)) y1 = y2 = 0;
  y[0] = y1;
  y[1] = y2;
}

// The three-direction normal equations by Cholesky; a direction whose pivot is
// not clearly positive is dropped.
__device__ inline void mr3_solve(const double *S, int m, double *y) {
  double A[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
  double g[3] = {S[6], S[7], S[8]};
  bool use[3] = {true, m == 2, true};
  double L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int j = 0; j < 3; ++j) {
    if (!use[j]) continue;
    double dj = A[j][j];
    for (int k = 0; k < j; ++k)
      if (use[k]) dj -= L[j][k] * L[j][k];
    if (!(dj > 1e-12 * A[j][j]) || !(A[j][j] > 0)) {
      use[j] = false;
      continue;
    }
    L[j][j] = sqrt(dj);
    for (int i = j + 1; i < 3; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k)
        if (use[k]) s -= L[i][k] * L[j][k];
      L[i][j] = s / L[j][j];
    }
  }
  double z[3] = {0, 0, 0}, x[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    if (!use[i]) continue;
    double s = g[i];
    for (int k = 0; k < i; ++k)
      if (use[k]) s -= L[i][k] * z[k];
    z[i] = s / L[i][i];
  }
  for (int i = 2; i >= 0; --i) {
    if (!use[i]) continue;
    double s = z[i];
    for (int k = i + 1; k < 3; ++k)
      if (use[k]) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
  for (int i = 0; i < 3; ++i) y[i] = isfinite(x[i]) ? x[i] : 0.0;
}

__device__ inline double wave_max(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
  return v;
}

template <typename T>
struct VT;
template <>
struct VT<double> {
  static constexpr const char *name = "f64";
};
template <>
struct VT<float> {
  static constexpr const char *name = "f32";
};

}  // namespace hho
