// Learned fine-level smoother (not in the paper): a two-layer network per face
// block maps a window of the residual to a correction of the face's velocity
// unknowns and of the pressure unknowns of its two cells (a cell takes the mean
// of its faces' predictions); it enters the smoothing step as one more search
// direction of the minimal-residual update, next to the Schwarz directions.
//
// Window of face F (n_in entries): for each side s of F (cells T_0 < T_1) the
// residual blocks of T_s's faces in the cell's face order, zero padded to Fm
// faces, then T_s's pressure residual; then a one-hot of F's position in T_0's
// and in T_1's face list.  The residual part is divided by its root mean square
// s_F (over 2 (Fm d p + t) entries) and the output is multiplied by s_F.
// Network: h = relu(W1 x + b1) (64 units), y = W2 h + b2 (d p + 2 t outputs),
// run on bfloat16 x, W1, h, W2 (rounded to nearest even) with FP32 sums on the
// matrix cores; biases and outputs FP32.  Master parameters are FP32
// [W1 | b1 | W2 | b2] (Adam updates them); their bfloat16 copies W1b [64][n_in16]
// and W2b [n_out16][64] (zero padded to multiples of 16) feed the products.
#include <algorithm>

#include "dev_common.h"
#include "device.h"

namespace hho {
namespace {


// one wavefront per face: gathers the window, its scale, and writes the scaled row
template <typename T>
__global__ void __launch_bounds__(kWave) k_mlp_windows(DTopo tp, MlpDims md, const T *__restrict__ r,
                                                        float *__restrict__ X, float *__restrict__ sc) {
  const int f = blockIdx.x;
  const int lane = threadIdx.x;
  const int side = md.Fm * md.dp + md.t;
  int cell[2], nfc[2], pos[2];
  for (int s = 0; s < 2; ++s) {
    cell[s] = tp.fcell[2 * f + s];
    nfc[s] = cell[s] >= 0 ? tp.cptr[cell[s] + 1] - tp.cptr[cell[s]] : 0;
    pos[s] = cell[s] >= 0 ? tp.floc[2 * f + s] : -1;
  }
  auto value = [&](int k) -> double {
    const int s = k / side, q = k % side;
    const int c = cell[s];
    if (c < 0) return 0.0;
    if (q < md.Fm * md.dp) {
      const int i = q / md.dp, j = q % md.dp;
      if (i >= nfc[s]) return 0.0;
      const int g = tp.cface[tp.cptr[c] + i];
      return (double)r[(int64_t)g * md.dp + j];
    }
    return (double)r[md.nface + (int64_t)c * md.t + (q - md.Fm * md.dp)];
  };
  double ss = 0;
  for (int k = lane; k < md.n_res; k += kWave) {
    const double v = value(k);
    ss += v * v;
  }
  ss = wave_sum(ss);
  ss = __shfl(ss, 0, kWave);
  const double s = sqrt(ss / md.n_res);
  const double inv = s > 0 ? 1.0 / s : 0.0;
  float *row = X + (int64_t)f * md.n_in;
  for (int k = lane; k < md.n_res; k += kWave) row[k] = (float)(value(k) * inv);
  for (int k = md.n_res + lane; k < md.n_in; k += kWave) {
    const int q = k - md.n_res, s_ = q / md.Fm, i = q % md.Fm;
    row[k] = (pos[s_] == i) ? 1.0f : 0.0f;
  }
  if (lane == 0) sc[f] = (float)s;
}

// targets (e_F, e_T0, e_T1) / s_F, e = xt - x (0 when s_F = 0 and for an absent T1)
__global__ void k_mlp_targets(DTopo tp, MlpDims md, const double *xt, const double *x, const float *sc, float *Tg) {
  const int64_t n = (int64_t)tp.nf * md.n_out;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(i / md.n_out), o = (int)(i % md.n_out);
    const float s = sc[f];
    int64_t src = -1;
    if (o < md.dp) {
      src = (int64_t)f * md.dp + o;
    } else {
      const int side = (o - md.dp) / md.t, q = (o - md.dp) % md.t;
      const int c = tp.fcell[2 * f + side];
      if (c >= 0) src = md.nface + (int64_t)c * md.t + q;
    }
    Tg[i] = (s > 0 && src >= 0) ? (float)((xt[src] - x[src]) / (double)s) : 0.0f;
  }
}

// bfloat16 copies of the weights for the matrix-core products
__global__ void k_mlp_pack(int n_in, int n_in16, int n_out, int n_out16, const float *prm, uint16_t *W1b,
                           uint16_t *W2b) {
  const float *W1 = prm, *W2 = W1 + (int64_t)kMlpHidden * n_in + kMlpHidden;
  const int64_t n1 = (int64_t)kMlpHidden * n_in16, n2 = (int64_t)n_out16 * kMlpHidden;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1 + n2; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n1) {
      const int h = (int)(i / n_in16), k = (int)(i % n_in16);
      W1b[i] = k < n_in ? to_bf16(W1[(int64_t)h * n_in + k]).bits : (uint16_t)0;
    } else {
      const int64_t j = i - n1;
      const int o = (int)(j / kMlpHidden), h = (int)(j % kMlpHidden);
      W2b[j] = o < n_out ? to_bf16(W2[(int64_t)o * kMlpHidden + h]).bits : (uint16_t)0;
    }
  }
}

typedef short v4bf16 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kMfmaRows = 64;  // rows per block: 16 per wavefront

// Forward pass on the matrix cores (16x16x16 bfloat16 products, FP32 sums):
// each wavefront takes 16 rows; layer 1 gives its 16 x 64 pre-activations Z
// (+ b1; written to Zout if not null), h = bf16(relu(Z)) goes through LDS to
// layer 2, Y = h W2^T + b2 for the 16 rows.  rows (optional) maps a row of the
// tile to the row of X it reads.
__global__ void __launch_bounds__(256) k_mlp_forward_mfma(int n, int n_in, int n_in16, int n_out, int n_out16,
                                                           const float *__restrict__ X, const int *__restrict__ rows,
                                                           const float *__restrict__ prm,
                                                           const uint16_t *__restrict__ W1b,
                                                           const uint16_t *__restrict__ W2b,
                                                           float *__restrict__ Zout, float *__restrict__ Y) {
  __shared__ uint16_t Hs[kMfmaRows][kMlpHidden + 4];
  const float *b1 = prm + (int64_t)kMlpHidden * n_in, *b2 = b1 + kMlpHidden + (int64_t)n_out * kMlpHidden;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int r16 = wave * 16;                          // the wave's rows in the block
  const int gi = blockIdx.x * kMfmaRows + r16 + lane % 16;  // row of the A fragment
  const int64_t src = gi < n ? (rows ? rows[gi] : gi) : -1;
  const float *xrow = src >= 0 ? X + src * n_in : nullptr;
  v4f acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < n_in16; kb += 16) {
    const int k0 = kb + 4 * (lane / 16);
    v4bf16 a;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + v;
      a[v] = (xrow && k < n_in) ? (short)to_bf16(xrow[k]).bits : (short)0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {  // hidden units 16 t .. 16 t + 15
      const uint16_t *w = W1b + (int64_t)(16 * t + lane % 16) * n_in16 + k0;
      v4bf16 b;
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = (short)w[v];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  // D layout: lane holds column lane % 16, rows 4 (lane / 16) + v
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r16 + 4 * (lane / 16) + v, h = 16 * t + lane % 16;
      const float z = acc[t][v] + b1[h];
      const int64_t g = (int64_t)blockIdx.x * kMfmaRows + row;
      if (Zout && g < n) Zout[g * kMlpHidden + h] = z;
      Hs[row][h] = to_bf16(z > 0.f ? z : 0.f).bits;
    }
  __syncthreads();
  for (int ob = 0; ob < n_out16; ob += 16) {
    v4f y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < kMlpHidden; kb += 16) {
      const int k0 = kb + 4 * (lane / 16);
      v4bf16 a, b;
      const uint16_t *w = W2b + (int64_t)(ob + lane % 16) * kMlpHidden + k0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        a[v] = (short)Hs[r16 + lane % 16][k0 + v];
        b[v] = (short)w[v];
      }
      y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, y, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t g = (int64_t)blockIdx.x * kMfmaRows + r16 + 4 * (lane / 16) + v;
      const int o = ob + lane % 16;
      if (g < n && o < n_out) Y[g * n_out + o] = y[v] + b2[o];
    }
  }
}

// z (level 0 layout): s_F y_F[:dp] on faces; on a cell T the mean over its faces
// F of s_F y_F[dp + side t + q], side = T's position in F's cell pair
template <typename T>
__global__ void k_mlp_scatter(DTopo tp, MlpDims md, int64_t N, const float *Y, const float *sc, T *z) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < md.nface) {
      const int64_t f = i / md.dp;
      z[i] = (T)(sc[f] * Y[f * md.n_out + i % md.dp]);
    } else {
      const int c = (int)((i - md.nface) / md.t), q = (int)((i - md.nface) % md.t);
      const int e0 = tp.cptr[c], e1 = tp.cptr[c + 1];
      float acc = 0;
      for (int e = e0; e < e1; ++e) {
        const int f = tp.cface[e];
        const int side = tp.fcell[2 * f] == c ? 0 : 1;
        acc += sc[f] * Y[(int64_t)f * md.n_out + md.dp + side * md.t + q];
      }
      z[i] = (T)(acc / (float)(e1 - e0));
    }
  }
}

// dY = (Y - T[rows]) / B and per-block partial sums of |Y - T|^2
__global__ void __launch_bounds__(kBlock) k_mlp_dy(int B, int n_out, const float *Y, const float *Tg,
                                                    const int *rows, float *dY, double *partial) {
  __shared__ double red[16];
  double acc = 0;
  const int64_t n = (int64_t)B * n_out;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / n_out, o = i % n_out;
    const int64_t src = rows ? rows[b] : b;
    const float dv = Y[i] - Tg[src * n_out + o];
    dY[i] = dv / (float)B;
    acc += (double)dv * dv;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// dZ = (dY W2b) .* (Z > 0), W2b the bfloat16 weights the forward pass used
__global__ void k_mlp_dz(int B, int n_out, const float *dY, const float *Z, const uint16_t *W2b, float *dZ) {
  const int64_t n = (int64_t)B * kMlpHidden;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / kMlpHidden, h = i % kMlpHidden;
    float s = 0;
    for (int o = 0; o < n_out; ++o) s += dY[b * n_out + o] * bf16_value(W2b[o * kMlpHidden + h]);
    dZ[i] = Z[i] > 0 ? s : 0.0f;
  }
}

// gradient of every parameter: one thread per parameter, sum over the batch in
// order, on the bfloat16-rounded inputs and activations the forward pass used
__global__ void k_mlp_wgrad(int B, int n_in, int n_out, const float *X, const int *rows, const float *Z,
                            const float *dZ, const float *dY, float *g) {
  const int64_t nW1 = (int64_t)kMlpHidden * n_in, nb1 = kMlpHidden, nW2 = (int64_t)n_out * kMlpHidden;
  const int64_t total = nW1 + nb1 + nW2 + n_out;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    float s = 0;
    if (p < nW1) {
      const int h = (int)(p / n_in), k = (int)(p % n_in);
      for (int b = 0; b < B; ++b) {
        const int64_t src = rows ? rows[b] : b;
        s += dZ[(int64_t)b * kMlpHidden + h] * (float)to_bf16(X[src * n_in + k]);
      }
    } else if (p < nW1 + nb1) {
      const int h = (int)(p - nW1);
      for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * kMlpHidden + h];
    } else if (p < nW1 + nb1 + nW2) {
      const int64_t q = p - nW1 - nb1;
      const int o = (int)(q / kMlpHidden), h = (int)(q % kMlpHidden);
      for (int b = 0; b < B; ++b) {
        const float z = Z[(int64_t)b * kMlpHidden + h];
        s += dY[(int64_t)b * n_out + o] * (float)to_bf16(z > 0 ? z : 0.0f);
      }
    } else {
      const int o = (int)(p - nW1 - nb1 - nW2);
      for (int b = 0; b < B; ++b) s += dY[(int64_t)b * n_out + o];
    }
    g[p] = s;
  }
}

// Adam (Kingma & Ba): bias-corrected first and second moments
__global__ void k_mlp_adam(int64_t n, float *prm, const float *g, float *m, float *v, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// batch rows from SplitMix64 (Steele, Lea & Flood 2014) of (seed, step, i)
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_mlp_rows(int B, int64_t n, uint64_t seed, int step, int *rows) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x)
    rows[i] = (int)(splitmix64(seed ^ splitmix64(((uint64_t)step << 32) | (uint64_t)i)) % (uint64_t)n);
}

// ---- three-direction minimal residual (the smoothing step with the learned direction)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mr3_dots(int64_t n, const T *w1, const T *w2, const T *w3, const T *r,
                                                      double *partial) {
  __shared__ double red[16];
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // a11 a12 a13 a22 a23 a33 g1 g2 g3
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x1 = w1[i], x2 = w2 ? (double)w2[i] : 0.0, x3 = w3[i], rr = r[i];
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
  for (int k = 0; k < 9; ++k) {
    const double s = block_sum(v[k], red);
    if (threadIdx.x == 0) partial[k * gridDim.x + blockIdx.x] = s;
  }
}

// Solves the 3x3 (or 2x2 without the second Schwarz direction) normal equations
__global__ void __launch_bounds__(kBlock) k_mr3_finish(int G, int m, const double *partial, double *y) {
  __shared__ double S[9];
  reduce_partials(partial, G, 9, S);
  if (threadIdx.x == 0) mr3_solve(S, m, y);
}

template <typename T>
__global__ void k_mr3_update(int64_t n, const double *y, const T *z1, const T *z2, const T *z3, const T *w1,
                             const T *w2, const T *w3, T *x, T *r) {
  const T y1 = (T)y[0], y2 = (T)y[1], y3 = (T)y[2];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T a2 = z2 ? z2[i] : (T)0, b2 = w2 ? w2[i] : (T)0;
    x[i] += y1 * z1[i] + y2 * a2 + y3 * z3[i];
    r[i] -= y1 * w1[i] + y2 * b2 + y3 * w3[i];
  }
}

inline int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192)); }

}  // namespace

int64_t mlp_param_count(const MlpDims &md) {
  return (int64_t)kMlpHidden * md.n_in + kMlpHidden + (int64_t)md.n_out * kMlpHidden + md.n_out;
}

template <typename T>
void launch_mlp_windows(const DTopo &tp, const MlpDims &md, const T *r, float *X, float *sc, hipStream_t s) {
  if (tp.nf == 0) return;
  hipLaunchKernelGGL((k_mlp_windows<T>), dim3(tp.nf), dim3(kWave), 0, s, tp, md, r, X, sc);
}
void launch_mlp_targets(const DTopo &tp, const MlpDims &md, const double *xt, const double *x, const float *sc,
                        float *Tg, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_targets, dim3(blocks_for((int64_t)tp.nf * md.n_out)), dim3(kBlock), 0, s, tp, md, xt, x,
                     sc, Tg);
}
void launch_mlp_pack(const MlpDims &md, const float *prm, uint16_t *W1b, uint16_t *W2b, hipStream_t s) {
  const int64_t n = (int64_t)kMlpHidden * md.n_in16 + (int64_t)md.n_out16 * kMlpHidden;
  hipLaunchKernelGGL(k_mlp_pack, dim3(blocks_for(n)), dim3(kBlock), 0, s, md.n_in, md.n_in16, md.n_out, md.n_out16,
                     prm, W1b, W2b);
}
void launch_mlp_forward(int n, const MlpDims &md, const float *X, const int *rows, const float *prm,
                        const uint16_t *W1b, const uint16_t *W2b, float *Z, float *Y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_forward_mfma, dim3((n + kMfmaRows - 1) / kMfmaRows), dim3(256), 0, s, n, md.n_in, md.n_in16,
                     md.n_out, md.n_out16, X, rows, prm, W1b, W2b, Z, Y);
}
template <typename T>
void launch_mlp_scatter(const DTopo &tp, const MlpDims &md, int64_t N, const float *Y, const float *sc, T *z,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_mlp_scatter<T>), dim3(blocks_for(N)), dim3(kBlock), 0, s, tp, md, N, Y, sc, z);
}
int launch_mlp_backward(int B, int n_in, int n_out, const float *X, const int *rows, const float *Tg,
                        const uint16_t *W2b, const float *Z, const float *Y, float *dY, float *dZ, float *g,
                        double *partial, hipStream_t s) {
  const int G = std::min(256, blocks_for((int64_t)B * n_out));
  hipLaunchKernelGGL(k_mlp_dy, dim3(G), dim3(kBlock), 0, s, B, n_out, Y, Tg, rows, dY, partial);
  hipLaunchKernelGGL(k_mlp_dz, dim3(blocks_for((int64_t)B * kMlpHidden)), dim3(kBlock), 0, s, B, n_out,
                     (const float *)dY, Z, W2b, dZ);
  const int64_t np = (int64_t)kMlpHidden * n_in + kMlpHidden + (int64_t)n_out * kMlpHidden + n_out;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for(np)), dim3(kBlock), 0, s, B, n_in, n_out, X, rows, Z,
                     (const float *)dZ, (const float *)dY, g);
  return G;
}
void launch_mlp_adam(int64_t n, float *prm, const float *g, float *m, float *v, float lr, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, prm, g, m, v, lr, c1, c2);
}
void launch_mlp_rows(int B, int64_t n, uint64_t seed, int step, int *rows, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_rows, dim3(blocks_for(B)), dim3(kBlock), 0, s, B, n, seed, step, rows);
}
template <typename T>
void launch_mr3(int64_t n, int m, const T *z1, const T *z2, const T *z3, const T *w1, const T *w2, const T *w3, T *x,
                T *r, double *partial, double *y, hipStream_t s) {
  const int G = reduce_blocks(n);
  hipLaunchKernelGGL((k_mr3_dots<T>), dim3(G), dim3(kBlock), 0, s, n, w1, m == 2 ? w2 : (const T *)nullptr, w3, r,
                     partial);
  hipLaunchKernelGGL(k_mr3_finish, dim3(1), dim3(kBlock), 0, s, G, m, (const double *)partial, y);
  hipLaunchKernelGGL((k_mr3_update<T>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, (const double *)y, z1,
                     m == 2 ? z2 : (const T *)nullptr, z3, w1, m == 2 ? w2 : (const T *)nullptr, w3, x, r);
}

#define HHO_INST(T)                                                                                             \
  template void launch_mlp_windows<T>(const DTopo &, const MlpDims &, const T *, float *, float *, hipStream_t); \
  template void launch_mlp_scatter<T>(const DTopo &, const MlpDims &, int64_t, const float *, const float *, T *, \
                                      hipStream_t);                                                               \
  template void launch_mr3<T>(int64_t, int, const T *, const T *, const T *, const T *, const T *, const T *, T *, \
                              T *, double *, double *, hipStream_t);
HHO_INST(double)
HHO_INST(float)
#undef HHO_INST

}  // namespace hho
