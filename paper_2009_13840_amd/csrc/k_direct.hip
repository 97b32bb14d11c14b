// Coarsest-level sparse direct solver: multifrontal elimination over the nested
// dissection tree of direct.h (the paper solves its 2D coarse problems directly,
// Section 5.2).
//
// Each front is a dense m x m matrix [F11 F12; F21 F22] (row-major) over its
// unknowns, the nfs it eliminates first.  Elimination applies the sweep operator
// to the nfs pivots: a pivot k turns a_kk into -1/a_kk, the rest of row and
// column k into a_kj / a_kk and a_ik / a_kk, and every other entry into
// a_ij - a_ik a_kj / a_kk; sweeping a set of pivots one by one equals sweeping
// them as a block, and the matrix stays symmetric.  Afterwards the front holds
// -F11^{-1} | F11^{-1} F12 over F21 F11^{-1} | F22 - F21 F11^{-1} F12, the last
// block being the update its parent adds to its own front.  The solves use the
// first three blocks as dense products:
//   forward (leaves up):  u = v2 - (F21 F11^{-1}) v1, passed to the parent;
//   backward (root down): x1 = F11^{-1} v1 - (F11^{-1} F12) x2, i.e. minus the
//                         front's first nfs rows times [v1; x2].
// Fronts of at most kNdSmall unknowns are swept by one block each, the front in
// its registers; larger ones in panels of kNdPanel pivots: one launch inverts
// the panel's pivot block and
// forms W = M_RP M_PP^{-1} by row chunks, the next updates the front's lower
// triangle by 64 x 64 tiles and mirrors it (M_RR -= W M_PR, M_RP = W,
// M_PR = W^T, M_PP = -M_PP^{-1}); the first panel's two launches also add the
// children's updates to what they read.
#include <mutex>

#include "dev_common.h"
#include "k_direct.h"

namespace hho {
namespace {

constexpr int kNdThreads = 256;
constexpr int kNdWaves = kNdThreads / kWave;
constexpr int kNdSweepThreads = 512;  // the sweeping kernels: eight waves
constexpr int kNdSolveThreads = kNdSolveRows / 16 * kWave;  // the solve kernels: 16 rows per wave
constexpr int kNdSweepWaves = kNdSweepThreads / kWave;
constexpr int kNdLd = kNdPanel + 1;  // padded row length of LDS tiles (no bank conflicts on transposed writes)

inline unsigned nd_grid(int64_t n) { return (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 65536); }

__device__ inline bool bad_pivot(double x) { return x == 0.0 || !isfinite(x); }

// 1 / x: the hardware reciprocal refined by two Newton steps (the pivot chain
// is latency-bound; a correctly rounded division costs twice as long)
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// operator entries into the (cleared) fronts: each lands in exactly one place
__global__ void __launch_bounds__(kBlock) k_nd_place(int64_t npair, const int64_t *src, const int64_t *dst,
                                                      const double *bsr, const double *cpl, const double *spp,
                                                      int64_t nb, int64_t ncpl, double *F) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npair; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = src[e];
    F[dst[e]] = s < nb ? bsr[s] : (s < nb + ncpl ? cpl[s - nb] : spp[s - nb - ncpl]);
  }
}

struct ChildRef {
  int f = -1, m = 0, nfs = 0;
  int64_t off = 0, voff = 0;
};

__device__ inline ChildRef child_ref(const NdDev &D, int F, int s) {
  ChildRef c;
  c.f = D.child[2 * F + s];
  if (c.f >= 0) {
    c.m = D.m[c.f];
    c.nfs = D.nfs[c.f];
    c.off = D.off[c.f];
    c.voff = D.voff[c.f];
  }
  return c;
}

// entry (ia, ib) of a child's update block
__device__ inline double child_u(const NdDev &D, const ChildRef &c, int ia, int ib) {
  return D.F[c.off + (int64_t)(c.nfs + ia) * c.m + c.nfs + ib];
}

// what the children pass to entry (a, b) of front F (child 0's, then child 1's)
__device__ inline double children_sum(const NdDev &D, const ChildRef (&ch)[2], int64_t dofo, int a, int b) {
  double v = 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (ch[s].f < 0) continue;
    const int ca = D.cmap[2 * (dofo + a) + s], cb = D.cmap[2 * (dofo + b) + s];
    if (ca >= 0 && cb >= 0) v += child_u(D, ch[s], ca, cb);
  }
  return v;
}

// Fronts of one height with at most kNdSmall (128) unknowns: one block each,
// the front held in registers (thread (w, lane) of the eight waves holds rows
// w + 8 u, u < 16, at columns lane and lane + 64); children's updates added
// while loading, then the nfs pivots swept one at a time.  The front stays
// symmetric, so the pivot column alone, passed through LDS (two buffers, one
// barrier per pivot), also gives the pivot row.
__global__ void __launch_bounds__(kNdSweepThreads) k_nd_small(NdDev D, const int32_t *fronts, int *err) {
  __shared__ double colk[2][kNdSmall];
  const int F = fronts[blockIdx.x];
  const int m = D.m[F], nfs = D.nfs[F];
  if (m == 0) return;
  const int64_t o = D.off[F], dofo = D.dofoff[F];
  const ChildRef c0 = child_ref(D, F, 0), c1 = child_ref(D, F, 1);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  int bmap0[2], bmap1[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int b = lane + kWave * t;
    bmap0[t] = (c0.f >= 0 && b < m) ? D.cmap[2 * (dofo + b)] : -1;
    bmap1[t] = (c1.f >= 0 && b < m) ? D.cmap[2 * (dofo + b) + 1] : -1;
  }
  double q[16][2];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = w + kNdSweepWaves * u;
    const int a0 = (c0.f >= 0 && a < m) ? D.cmap[2 * (dofo + a)] : -1;
    const int a1 = (c1.f >= 0 && a < m) ? D.cmap[2 * (dofo + a) + 1] : -1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int b = lane + kWave * t;
      double v = 0.0;
      if (a < m && b < m) {
        v = D.F[o + (int64_t)a * m + b];
        if (a0 >= 0 && bmap0[t] >= 0) v += child_u(D, c0, a0, bmap0[t]);
        if (a1 >= 0 && bmap1[t] >= 0) v += child_u(D, c1, a1, bmap1[t]);
      }
      q[u][t] = v;
    }
  }
  for (int k = 0; k < nfs; ++k) {
    double *ck = colk[k & 1];
    if (lane == (k & (kWave - 1))) {  // these lanes hold column k (k is the same in every thread)
      if (k >= kWave) {
#pragma unroll
        for (int u = 0; u < 16; ++u) ck[w + kNdSweepWaves * u] = q[u][1];
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) ck[w + kNdSweepWaves * u] = q[u][0];
      }
    }
    __syncthreads();
    const double piv = ck[k];
    if (bad_pivot(piv) && threadIdx.x == 0) err[0] = F + 1;
    const double inv = recip(piv);
    const double rb0 = ck[lane] * inv, rb1 = ck[min(lane + kWave, kNdSmall - 1)] * inv;
    double ca[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) ca[u] = ck[w + kNdSweepWaves * u];
    // every entry as if off the pivot row and column, then the pivot column (one
    // lane of each wave) and the pivot row (one wave) overwritten
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      q[u][0] -= ca[u] * rb0;
      q[u][1] -= ca[u] * rb1;
    }
    if (lane == (k & (kWave - 1))) {
      if (k >= kWave) {
#pragma unroll
        for (int u = 0; u < 16; ++u) q[u][1] = ca[u] * inv;
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) q[u][0] = ca[u] * inv;
      }
    }
    if (w == (k & (kNdSweepWaves - 1))) {
      const int ks = k / kNdSweepWaves;
      const double rv0 = lane == k ? -inv : rb0, rv1 = lane + kWave == k ? -inv : rb1;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        q[u][0] = u == ks ? rv0 : q[u][0];
        q[u][1] = u == ks ? rv1 : q[u][1];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = w + kNdSweepWaves * u;
    if (a >= m) continue;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int b = lane + kWave * t;
      if (b < m) D.F[o + (int64_t)a * m + b] = q[u][t];
    }
  }
}

// Panel [k0, k0 + nb) of a larger front: the pivot block swept in registers
// (thread (w, lane) of the block's eight waves holds entries (w + 8 u, lane),
// u < 8; the block stays symmetric, so its pivot column also gives the pivot
// row; every chunk's block does it, the first stores the inverse), then for the
// chunk's rows the panel columns as they are (S1) and W = S1 M_PP^{-1} (rows
// outside the panel).  Scratch of the front:
// [M_PP^{-1} (64 x 64) | S1 (m x 64) | W (m x 64)].
__global__ void __launch_bounds__(kNdSweepThreads) k_nd_panel(NdDev D, const int32_t *chunks, int k0, int *err) {
  extern __shared__ double lds_panel[];
  double *Q = lds_panel;                       // M_PP^{-1}, rows of kNdLd
  double *Sr = Q + kNdPanel * kNdLd;           // the chunk's panel columns
  double *colk = Sr + kNdChunk * kNdLd;        // pivot column, two buffers
  const int F = chunks[2 * blockIdx.x], r0 = chunks[2 * blockIdx.x + 1];
  const int m = D.m[F], nfs = D.nfs[F];
  if (k0 >= nfs) return;
  const int nb = min(kNdPanel, nfs - k0);
  const double *M = D.F + D.off[F];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  // the first panel adds the children's updates to the entries it reads (the
  // first update launch adds them to the rest of the front)
  const ChildRef ch[2] = {child_ref(D, F, 0), child_ref(D, F, 1)};
  const bool ext = k0 == 0 && (ch[0].f >= 0 || ch[1].f >= 0);
  const int64_t dofo = D.dofoff[F];
  constexpr int U = kNdPanel / kNdSweepWaves;
  double q[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int a = w + kNdSweepWaves * u;
    double v = 0.0;
    if (a < nb && lane < nb) {
      v = M[(int64_t)(k0 + a) * m + k0 + lane];
      if (ext) v += children_sum(D, ch, dofo, k0 + a, k0 + lane);
    }
    q[u] = v;
  }
  for (int k = 0; k < nb; ++k) {
    double *ck = colk + (k & 1) * kNdPanel;
    if (lane == k) {
#pragma unroll
      for (int u = 0; u < U; ++u) ck[w + kNdSweepWaves * u] = q[u];
    }
    __syncthreads();
    const double piv = ck[k];
    if (bad_pivot(piv) && threadIdx.x == 0) err[0] = F + 1;
    const double inv = recip(piv);
    const double rb = ck[lane] * inv;
    double ca[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ca[u] = ck[w + kNdSweepWaves * u];  // all reads in flight at once
    // every entry as if off the pivot row and column, then the pivot column (one
    // lane of each wave) and the pivot row (one wave) overwritten
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] -= ca[u] * rb;
    if (lane == k) {
#pragma unroll
      for (int u = 0; u < U; ++u) q[u] = ca[u] * inv;
    }
    if (w == (k & (kNdSweepWaves - 1))) {
      const int ks = k / kNdSweepWaves;
      const double rv = lane == k ? -inv : rb;
#pragma unroll
      for (int u = 0; u < U; ++u) q[u] = u == ks ? rv : q[u];
    }
  }
  // q = -M_PP^{-1}
#pragma unroll
  for (int u = 0; u < U; ++u) Q[(w + kNdSweepWaves * u) * kNdLd + lane] = -q[u];
  double *Sc = D.S + D.soff[F];
  double *S1 = Sc + kNdPanel * kNdPanel, *W = S1 + (int64_t)m * kNdPanel;
  if (r0 == 0)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int a = w + kNdSweepWaves * u;
      if (a < nb && lane < nb) Sc[a * kNdPanel + lane] = -q[u];
    }
  const int nr = min(kNdChunk, m - r0);
  for (int i = w; i < nr; i += kNdSweepWaves) {
    double v = 0.0;
    if (lane < nb) {
      v = M[(int64_t)(r0 + i) * m + k0 + lane];
      if (ext) v += children_sum(D, ch, dofo, r0 + i, k0 + lane);
    }
    Sr[i * kNdLd + lane] = v;
    if (lane < nb) S1[(int64_t)(r0 + i) * kNdPanel + lane] = v;
  }
  __syncthreads();
  // W = Sr M_PP^{-1}: thread (ty, tx) forms rows ty + 32 r, columns tx + 16 c
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[2][4] = {};
  for (int p = 0; p < nb; ++p) {
    double a[2], b[4];
#pragma unroll
    for (int r = 0; r < 2; ++r) a[r] = Sr[(ty + 32 * r) * kNdLd + p];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = Q[p * kNdLd + tx + 16 * c];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int i = ty + 32 * r, row = r0 + i;
    if (i >= nr || (row >= k0 && row < k0 + nb)) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int pc = tx + 16 * c;
      if (pc < nb) W[(int64_t)row * kNdPanel + pc] = acc[r][c];
    }
  }
}

// The panel's sweep applied to one 64 x 64 tile of the lower triangle of a
// larger front, and its transpose written to the mirror tile (the front is
// symmetric).  Thread (ty, tx) owns rows ty + 16 r and columns tx + 16 c (r, c < 4).
__global__ void __launch_bounds__(kNdThreads) k_nd_update(NdDev D, const int32_t *tiles, int k0) {
  extern __shared__ double lds_update[];
  double *Wt = lds_update;                 // Wt[p * kNdLd + i]: W of the tile's rows, transposed
  double *St = Wt + kNdPanel * kNdLd;      // St[p * kNdLd + j]: S1 of the tile's columns, transposed
  const int F = tiles[3 * blockIdx.x], r0 = tiles[3 * blockIdx.x + 1], q0 = tiles[3 * blockIdx.x + 2];
  const int m = D.m[F], nfs = D.nfs[F];
  if (k0 > 0 && k0 >= nfs) return;
  const int nb = max(0, min(kNdPanel, nfs - k0));  // 0: a front with no own unknown, only extended
  const ChildRef ch[2] = {child_ref(D, F, 0), child_ref(D, F, 1)};
  const bool ext = k0 == 0 && (ch[0].f >= 0 || ch[1].f >= 0);
  if (nb == 0 && !ext) return;
  const int64_t dofo = D.dofoff[F];
  const double *Sc = D.S + D.soff[F];
  const double *S1 = Sc + kNdPanel * kNdPanel, *W = S1 + (int64_t)m * kNdPanel;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  for (int i = w; i < kNdTile; i += kNdWaves) {
    Wt[lane * kNdLd + i] = (r0 + i < m && lane < nb) ? W[(int64_t)(r0 + i) * kNdPanel + lane] : 0.0;
    St[lane * kNdLd + i] = (q0 + i < m && lane < nb) ? S1[(int64_t)(q0 + i) * kNdPanel + lane] : 0.0;
  }
  __syncthreads();
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int p = 0; p < nb; ++p) {
    double a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = Wt[p * kNdLd + ty + 16 * r];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = St[p * kNdLd + tx + 16 * c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
  }
  double *M = D.F + D.off[F];
  const bool mirror = r0 != q0;
  __syncthreads();  // Wt / St no longer read: the tile's new values are staged in Wt
  double *T = Wt;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = r0 + ty + 16 * r;
    const bool iP = row >= k0 && row < k0 + nb;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int cl = q0 + tx + 16 * c;
      if (row >= m || cl >= m) continue;
      const bool jP = cl >= k0 && cl < k0 + nb;
      double &x = M[(int64_t)row * m + cl];
      double nv;
      if (!iP && !jP)
        nv = (ext ? x + children_sum(D, ch, dofo, row, cl) : x) - acc[r][c];
      else if (!iP)
        nv = W[(int64_t)row * kNdPanel + (cl - k0)];
      else if (!jP)
        nv = W[(int64_t)cl * kNdPanel + (row - k0)];
      else
        nv = -Sc[(row - k0) * kNdPanel + (cl - k0)];
      x = nv;
      if (mirror) T[(ty + 16 * r) * kNdLd + tx + 16 * c] = nv;
    }
  }
  if (!mirror) return;
  __syncthreads();
  // the front stays symmetric: the mirror tile (rows q0.., columns r0..) is the transpose
  for (int i = w; i < kNdTile; i += kNdWaves) {
    if (q0 + i >= m || r0 + lane >= m) continue;
    M[(int64_t)(q0 + i) * m + r0 + lane] = T[lane * kNdLd + i];
  }
}

// Forward elimination over one height, one block per kNdSolveRows rows of a front:
// v = the front's own unknowns of b (minus coef times the null vector) plus what
// its children passed up; the first chunk keeps v1 = v[0, nfs) for the backward
// pass and every chunk writes u = v2 - (F21 F11^{-1}) v1 for its update rows.
__global__ void __launch_bounds__(kNdSolveThreads) k_nd_fwd(NdDev D, const int32_t *chunks, const double *b,
                                                        int64_t nface, int t, const double *zmean,
                                                        const double *coef) {
  extern __shared__ double v[];
  const int F = chunks[2 * blockIdx.x], r0 = chunks[2 * blockIdx.x + 1];
  const int m = D.m[F], nfs = D.nfs[F];
  const int64_t dofo = D.dofoff[F];
  const ChildRef c0 = child_ref(D, F, 0), c1 = child_ref(D, F, 1);
  for (int a = threadIdx.x; a < m; a += kNdSolveThreads) {
    double x = 0;
    if (a < nfs) {
      const int64_t g = D.dof[dofo + a];
      x = b[g];
      if (coef && g >= nface && (g - nface) % t == 0) {
        const int64_t T = (g - nface) / t;
        x -= coef[D.cseg[T]] * zmean[T];
      }
    }
    if (c0.f >= 0) {
      const int ca = D.cmap[2 * (dofo + a)];
      if (ca >= 0) x += D.V[c0.voff + c0.nfs + ca];
    }
    if (c1.f >= 0) {
      const int ca = D.cmap[2 * (dofo + a) + 1];
      if (ca >= 0) x += D.V[c1.voff + c1.nfs + ca];
    }
    v[a] = x;
  }
  __syncthreads();
  double *Vf = D.V + D.voff[F];
  if (r0 == 0)
    for (int a = threadIdx.x; a < nfs; a += kNdSolveThreads) Vf[a] = v[a];
  // each wave takes 16 of the chunk's rows at once (16 loads in flight per lane)
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lo = max(r0 + 16 * w, nfs), hi = min(r0 + 16 * w + 16, m);
  if (lo >= hi) return;
  const int nrw = hi - lo;
  const double *M = D.F + D.off[F] + (int64_t)lo * m;
  double acc[16] = {};
  int64_t ro[16];  // row offsets, rows past the chunk clamped to its last (read, never written)
#pragma unroll
  for (int r = 0; r < 16; ++r) ro[r] = (int64_t)min(r, nrw - 1) * m;
  for (int c = lane; c < nfs; c += kWave) {
    double mv[16];  // the 16 loads issued before any is used
#pragma unroll
    for (int r = 0; r < 16; ++r) mv[r] = __builtin_nontemporal_load(M + ro[r] + c);
    __builtin_amdgcn_sched_barrier(0);  // keep the 16 loads ahead of their uses
    const double vc = v[c];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += mv[r] * vc;
  }
  wave_multi_sum<16>(acc);  // acc[0]: the sum of row lane / 4
  const int r = lane >> 2;
  if ((lane & 3) == 0 && r < nrw) Vf[lo + r] = v[lo + r] - acc[0];
}

// Backward substitution over one height (root first): x1 = -[front row] . [v1; x2]
// for the chunk's rows among the front's own unknowns.
__global__ void __launch_bounds__(kNdSolveThreads) k_nd_bwd(NdDev D, const int32_t *chunks, double *x) {
  extern __shared__ double y[];
  const int F = chunks[2 * blockIdx.x], r0 = chunks[2 * blockIdx.x + 1];
  const int m = D.m[F], nfs = D.nfs[F];
  if (r0 >= nfs) return;
  const int64_t dofo = D.dofoff[F];
  const double *Vf = D.V + D.voff[F];
  for (int a = threadIdx.x; a < m; a += kNdSolveThreads) y[a] = a < nfs ? Vf[a] : x[D.dof[dofo + a]];
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int lo = r0 + 16 * w, hi = min(r0 + 16 * w + 16, nfs);
  if (lo >= hi) return;
  const int nrw = hi - lo;
  const double *M = D.F + D.off[F] + (int64_t)lo * m;
  double acc[16] = {};
  int64_t ro[16];  // row offsets, rows past the chunk clamped to its last (read, never written)
#pragma unroll
  for (int r = 0; r < 16; ++r) ro[r] = (int64_t)min(r, nrw - 1) * m;
  for (int c = lane; c < m; c += kWave) {
    double mv[16];  // the 16 loads issued before any is used
#pragma unroll
    for (int r = 0; r < 16; ++r) mv[r] = __builtin_nontemporal_load(M + ro[r] + c);
    __builtin_amdgcn_sched_barrier(0);  // keep the 16 loads ahead of their uses
    const double yc = y[c];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += mv[r] * yc;
  }
  wave_multi_sum<16>(acc);  // acc[0]: the sum of row lane / 4
  const int r = lane >> 2;
  if ((lane & 3) == 0 && r < nrw) x[D.dof[dofo + lo + r]] = -acc[0];
}

// per member (one block each): coef = (z . b) / (z . z), z the member's
// constant-pressure null vector (its cells' mean modes)
__global__ void __launch_bounds__(1024) k_nd_proj_in(const int64_t *segp, int64_t nface, int t, const double *zmean,
                                                      const double *b, double *coef) {
  __shared__ double red[16];
  const int64_t c0 = segp[blockIdx.x], c1 = segp[blockIdx.x + 1];
  double zb = 0, zz = 0;
  for (int64_t T = c0 + threadIdx.x; T < c1; T += blockDim.x) {
    zb += zmean[T] * b[nface + T * t];
    zz += zmean[T] * zmean[T];
  }
  zb = block_sum(zb, red);
  __syncthreads();
  zz = block_sum(zz, red);
  if (threadIdx.x == 0) coef[blockIdx.x] = zb / zz;
}

// per member (one block each): its pinned unknown set to zero, then
// x <- x - ((z . x) / (z . z)) z on its cells
__global__ void __launch_bounds__(1024) k_nd_proj_out(const int64_t *segp, const int64_t *pins, int64_t nface, int t,
                                                       const double *zmean, double *x) {
  __shared__ double red[16];
  __shared__ double c;
  const int64_t c0 = segp[blockIdx.x], c1 = segp[blockIdx.x + 1], pin = pins[blockIdx.x];
  double zx = 0, zz = 0;
  for (int64_t T = c0 + threadIdx.x; T < c1; T += blockDim.x) {
    const int64_t i = nface + T * t;
    zx += zmean[T] * (i == pin ? 0.0 : x[i]);
    zz += zmean[T] * zmean[T];
  }
  zx = block_sum(zx, red);
  __syncthreads();
  zz = block_sum(zz, red);
  if (threadIdx.x == 0) c = zx / zz;
  __syncthreads();
  for (int64_t T = c0 + threadIdx.x; T < c1; T += blockDim.x) {
    const int64_t i = nface + T * t;
    x[i] = (i == pin ? 0.0 : x[i]) - c * zmean[T];
  }
}

void reserve_lds(const void *fn, std::once_flag &once, hipError_t &attr) {
  std::call_once(once, [&] {
    attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLdsBytes - 1024));
  });
  if (attr != hipSuccess) fail(HHO_E_DEVICE, "sparse direct coarse solver: cannot reserve LDS");
}

}  // namespace

void launch_nd_factor(const NdHost &H, const NdDev &D, const DLevel<double> &L, int64_t nb, int64_t ncpl,
                      int *err, hipStream_t s) {
  static std::once_flag once_p, once_u;
  static hipError_t attr_p = hipSuccess, attr_u = hipSuccess;
  reserve_lds((const void *)k_nd_panel, once_p, attr_p);
  reserve_lds((const void *)k_nd_update, once_u, attr_u);
  const size_t lds_p = ((size_t)(kNdPanel + kNdChunk) * kNdLd + 2 * kNdPanel) * sizeof(double);
  const size_t lds_u = 2 * (size_t)kNdPanel * kNdLd * sizeof(double);
  launch_fill<double>(H.total, 0.0, D.F, s);
  if (D.npair > 0)
    hipLaunchKernelGGL(k_nd_place, dim3(nd_grid(D.npair)), dim3(kBlock), 0, s, D.npair, D.src, D.dst, L.bsr, L.cpl,
                       L.spp, nb, ncpl, D.F);
  for (int h = 0; h < H.nheight; ++h) {
    const int nfr = H.hptr[h + 1] - H.hptr[h];
    if (nfr == 0 || H.hmaxm[h] == 0) continue;
    if (!H.big[h]) {
      hipLaunchKernelGGL(k_nd_small, dim3(nfr), dim3(kNdSweepThreads), 0, s, D, D.hfront + H.hptr[h], err);
      continue;
    }
    const int ntile = H.tptr[h + 1] - H.tptr[h], nch = H.cptr[h + 1] - H.cptr[h];
    const int32_t *tiles = D.tiles + 3 * (int64_t)H.tptr[h], *chunks = D.chunks + 2 * (int64_t)H.cptr[h];
    // (the first panel's two launches also add the children's updates)
    for (int k0 = 0; k0 < std::max(H.hmaxnfs[h], 1); k0 += kNdPanel) {
      hipLaunchKernelGGL(k_nd_panel, dim3(nch), dim3(kNdSweepThreads), lds_p, s, D, chunks, k0, err);
      hipLaunchKernelGGL(k_nd_update, dim3(ntile), dim3(kNdThreads), lds_u, s, D, tiles, k0);
    }
  }
}

void launch_nd_solve(const NdHost &H, const NdDev &D, int64_t nface, int t, const double *zmean, const double *b,
                     double *x, hipStream_t s, KernelProbe *probe) {
  static std::once_flag once_f, once_b;
  static hipError_t attr_f = hipSuccess, attr_b = hipSuccess;
  reserve_lds((const void *)k_nd_fwd, once_f, attr_f);
  reserve_lds((const void *)k_nd_bwd, once_b, attr_b);
  const bool pin = !H.pins.empty() && H.pins[0] >= 0;  // every member has its null space, or none
  const int nsegp = (int)H.pins.size();
  if (pin) hipLaunchKernelGGL(k_nd_proj_in, dim3(nsegp), dim3(1024), 0, s, D.segp, nface, t, zmean, b, D.coef);
  for (int h = 0; h < H.nheight; ++h) {
    const int nch = H.scptr[h + 1] - H.scptr[h];
    if (nch == 0) continue;
    const size_t lds = (size_t)H.hmaxm[h] * sizeof(double);
    const int32_t *ch = D.schunks + 2 * (int64_t)H.scptr[h];
    const double *cf = pin ? (const double *)D.coef : nullptr;
    HHO_PROBED(probe, HHO_PROBE_DIRECT_FWD, h, s,
               HHO_LAUNCH(k_nd_fwd, dim3(nch), dim3(kNdSolveThreads), lds, s, D, ch, b, nface, t, zmean, cf));
  }
  for (int h = H.nheight - 1; h >= 0; --h) {
    const int nch = H.scptr[h + 1] - H.scptr[h];
    if (nch == 0) continue;
    const size_t lds = (size_t)H.hmaxm[h] * sizeof(double);
    const int32_t *ch = D.schunks + 2 * (int64_t)H.scptr[h];
    HHO_PROBED(probe, HHO_PROBE_DIRECT_BWD, h, s,
               HHO_LAUNCH(k_nd_bwd, dim3(nch), dim3(kNdSolveThreads), lds, s, D, ch, x));
  }
  if (pin) hipLaunchKernelGGL(k_nd_proj_out, dim3(nsegp), dim3(1024), 0, s, D.segp, D.pins, nface, t, zmean, x);
}

}  // namespace hho
