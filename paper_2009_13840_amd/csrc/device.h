// Device data structures and kernel launch wrappers of the HHO library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hho {

constexpr int kMaxRestartH = 64;

// Mesh topology on the device (int32 indices).
struct DTopo {
  int d;
  int nc, nf;
  int64_t ncf;             // cptr[nc]: number of (cell, face) entries
  int64_t nnzb;            // number of face blocks
  const int32_t *cptr;     // [nc+1] cell -> first entry of its face list
  const int32_t *cface;    // [cptr[nc]] faces of each cell
  const int32_t *fcell;    // [2*nf] adjacent cells (second = -1 on the boundary)
  const int32_t *floc;     // [2*nf] position of the face in each cell's list
  const int32_t *rowptr;   // [nf+1] face-block sparse rows
  const int32_t *col;      // [nnzb] block columns (faces), sorted per row
  const int32_t *mirror;   // [nnzb] index of the block (col, row) of each block (row, col)
  const int32_t *blksrc;   // [6*nnzb] (cell, i, j) of the <= 2 cell blocks summed into each block
  const int64_t *pairoff;  // [nc+1] prefix sum of card(F_T)^2
  const int32_t *pairblk;  // [pairoff[nc]] block index of the local pair (i, j) of each cell
  const double *zmean;     // [nc] |T|^{1/2}: mean-mode coefficient of the constant pressure
  int max_faces;           // largest card(F_T)
};

constexpr int kPatchMaxRows = 256;  // face rows of a patch inverse (one component block for v-cond)
constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS of one CDNA4 compute unit

// One level of the operator: face-block rows plus cell-local couplings.
//  v-cond:   bsr  [nnzb][p][p] scalar blocks (act on every velocity component),
//            cpl  [cptr*d*p*t] cell coupling S_dT, rows (face i, comp c, mode r), cols q,
//            spp  [nc][t][t]   S_TT.
//  v&p-cond: bsr  [nnzb][d*p][d*p] full blocks, cpl [cptr*d*p] mean-pressure coupling, spp unused.
// Operator values are stored as Sto and the smoother's factors as StoP (T; or
// bf16 with T = float: read as float).
template <typename T, typename Sto = T, typename StoP = Sto>
struct DLevel {
  int cond;  // 1 v, 2 vp
  int p, t;  // face modes, pressure modes per cell
  int64_t nface, N;  // face-part length nf*d*p, total length
  const Sto *bsr, *cpl, *spp;
  // smoother patches
  const StoP *sinv;  // v: [pairoff*p*p] s_P^{-1}; vp: [pairoff*(d p)^2] S_P^{-1}; each cell's
                  // slot holds the lower triangle packed by rows (i (i+1)/2 + j, i >= j)
  const StoP *xinv;  // v: [nc][t][t] pressure Schur inverse; vp: [cptr*d*p] g = S_P^{-1} b
  const StoP *sig;   // vp: [nc] 1 / (b^T S_P^{-1} b)
  int block = 0;  // threads per block of the operator kernels (0: default), chosen by the autotuner
  const int *skip = nullptr;  // lowest-degree operator kernels return at once while *skip != 0 (device flag)
};

// ---- setup kernels (FP64)
size_t condense_lds_bytes(int d, int cond, int nT, int nF, int max_faces);
size_t patch_lds_bytes(int d, int cond, int p, int t, int max_faces);
// stage32 (may be null): the V-cycle copy's face blocks formed by the matrix-core
// bfloat16 product (FP32, laid out as stage)
void launch_condense(const DTopo &tp, int cond, int nT, int nF, const double *rec, const int64_t *roff,
                     double *stage, double *cpl, double *spp, double *rhs_stage, double *rhs_p, int *err,
                     hipStream_t s, size_t lds, float *stage32 = nullptr);
// face blocks of the V-cycle copy from stage32 (sum of <= 2 cell blocks in FP32)
template <typename Tout>
void launch_assemble32(const DTopo &tp, int cond, int nF, int64_t nnzb, const float *stage32, Tout *bsr,
                       hipStream_t s);
// Cell unknowns from the solved globally coupled ones x (level-0 layout):
// cu [nc][d*nT] velocities (component-major), cp [nc][nT] full pressures.
size_t recover_lds_bytes(int d, int nT, int nF, int max_faces);
void launch_recover(const DTopo &tp, int cond, int nT, int nF, const double *rec, const int64_t *roff,
                    const double *x, double *cu, double *cp, int *err, hipStream_t s, size_t lds);
void launch_assemble(const DTopo &tp, int cond, int nF, int64_t nnzb, const double *stage, double *bsr,
                     const double *rhs_stage, double *rhs, hipStream_t s);
void launch_extract(const DTopo &tp, int cond, int64_t nnzb, int p0, int t0, int p1, int t1, const double *bsr0,
                    const double *cpl0, const double *spp0, double *bsr1, double *cpl1, double *spp1, hipStream_t s);
// threads: threads per cell of the LDS-resident variant (0: chosen from the patch size)
void launch_patch_setup(const DTopo &tp, int cond, int p, int t, const double *bsr, const double *cpl,
                        const double *spp, double *sinv, double *xinv, double *sig, double *scratch, int *err,
                        hipStream_t s, size_t lds, int threads = 0);
template <typename Tout, typename Tin>
void launch_convert(const Tin *in, Tout *out, int64_t n, hipStream_t s);

// ---- dense coarse solver (FP64)
void launch_densify(const DTopo &tp, const DLevel<double> &L, int border, double *D, int64_t ld, hipStream_t s);
void launch_eye_right(double *D, int64_t n, int64_t ld, hipStream_t s);
void launch_gj_step(double *D, int64_t n, int64_t ld, int64_t k, double *colbuf, int *err, hipStream_t s);
void launch_dense_matvec(const double *Dinv, int64_t n, int64_t ld, int border, const double *x, double *y,
                         hipStream_t s);

// ---- solve kernels
size_t precond_lds_bytes(int d, int cond, int p, int t, int max_faces, size_t elem);
int reduce_blocks(int64_t n);
// y = S x (face rows and cell rows); if xs1 != null the face part of x is the sum of
// two slot vectors x (slot 0) and xs1 (slot 1), and xsum (if not null) receives it.
template <typename T, typename Sto, typename StoP>
void launch_spmv(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *x, const T *xs1, T *xsum, T *y, hipStream_t s);
// Compile-time-sized variants of the two calls above (b != null: residual form);
// false when no variant matches the level's block sizes.
template <typename T, typename Sto, typename StoP>
bool launch_spmv_fixed(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *x, const T *xs1, T *xsum, const T *b, T *y,
                       hipStream_t s);
// r = b - S x
template <typename T, typename Sto, typename StoP>
void launch_residual(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *b, const T *x, T *r, hipStream_t s);
// Schwarz preconditioner: face part in two slots (z: slot 0, zs1: slot 1), cells in z.
// If scale != null the input is scale[0]*r and v (if not null) receives that scaled vector.
template <typename T, typename Sto, typename StoP>
void launch_precond(const DTopo &tp, const DLevel<T, Sto, StoP> &L, const T *r, const double *scale, T *v, T *z, T *zs1,
                    int max_faces, hipStream_t s);
template <typename T>
void launch_combine(int64_t nface, const T *zs1, T *z, hipStream_t s);
// restriction of a level vector to the next coarser level (truncation) and prolongation-add
template <typename Tc, typename Tf>
void launch_restrict(int d, int nf, int nc, int pf, int tf, int pc, int tc, const Tf *xf, Tc *xc, hipStream_t s);
template <typename Tc, typename Tf>
void launch_prolong_add(int d, int nf, int nc, int pf, int tf, int pc, int tc, const Tc *xc, Tf *xf,
                        hipStream_t s);

// Smoother: minimal residual over span{z1, z2} (the GMRES(2) iterate):
//   G = [w1 w2]^T [w1 w2], g = [w1 w2]^T r, y = G^{-1} g, x += Z y, r -= W y.
template <typename T>
void launch_mr2_dots(int64_t n, int m, const T *w1, const T *w2, const T *r, double *partial, double *y,
                     hipStream_t s);
template <typename T>
void launch_mr2_update(int64_t n, int m, const double *y, const T *z1, const T *z2, const T *w1, const T *w2,
                       T *x, T *r, hipStream_t s);

struct GmresState;
template <typename T>
void launch_norm_init(int64_t n, const T *r, double *partial, GmresState *st, int which, hipStream_t s);
template <typename T>
void launch_scale(int64_t n, const T *x, const double *scale, T *y, hipStream_t s);
// Arnoldi step j (Section 3.3) on the basis V (columns of length n, stride ldv):
// dots: h1 = V^T w;  update pass 1: w -= V h1, h2 = V^T w;  update pass 2:
// w -= V h (h2 when cgs2, else h1), H[:, j] = h1 (+ h2), Givens rotation,
// residual estimate and convergence flag in *st.
template <typename T>
void launch_arnoldi_dots(int64_t n, int j, const T *V, int64_t ldv, const T *w, double *partial, GmresState *st,
                         hipStream_t s);
template <typename T>
void launch_arnoldi_update(int64_t n, int j, const T *V, int64_t ldv, T *w, double *partial, GmresState *st,
                           int pass, int cgs2, hipStream_t s);
// Classical Gram-Schmidt once, fused: h1 = V^T w and |w|^2 in one pass, the
// Hessenberg column (new norm |w|^2 - |h1|^2), Givens and residual estimate, then
// V_{j+1} = (w - V h1) / h_{j+1,j} written in one more pass (3 launches).
template <typename T>
void launch_arnoldi_cgs1(int64_t n, int j, T *V, int64_t ldv, const T *w, double *partial, GmresState *st,
                         hipStream_t s);
void launch_gmres_solve_ls(GmresState *st, hipStream_t s);
template <typename T>
void launch_gmres_combine(int64_t n, const T *Z, int64_t ldz, const GmresState *st, T *x, hipStream_t s);
template <typename T>
void launch_dot(int64_t n, const T *a, const T *b, double *partial, double *out, hipStream_t s);
// y += sign * alpha[0] / alpha[1] * x
template <typename T>
void launch_axpy_ratio(int64_t n, const double *alpha, double sign, const T *x, T *y, hipStream_t s);
template <typename T>
void launch_fill(int64_t n, T v, T *x, hipStream_t s);
template <typename T>
void launch_copy(int64_t n, const T *x, T *y, hipStream_t s);

// ---- learned smoother (k_mlp.hip)
constexpr int kMlpHidden = 64;
constexpr int kMlpMaxBatch = 4096;
constexpr int kMlpMaxSteps = 100000;
struct MlpDims {
  int d, p, t, Fm, dp, n_res, n_in, n_out;  // n_out = d p + 2 t: face velocity, then the two cells' pressures
  int n_in16, n_out16;                      // n_in, n_out rounded up to multiples of 16 (matrix-core tiles)
  int64_t nface;  // offset of the cell part of a level-0 vector
};
int64_t mlp_param_count(const MlpDims &md);
// window of every face of r -> X [nf][n_in] (FP32, scaled), sc [nf] (scales)
template <typename T>
void launch_mlp_windows(const DTopo &tp, const MlpDims &md, const T *r, float *X, float *sc, hipStream_t s);
// targets (xt - x) on F, T_0, T_1, divided by s_F -> Tg [nf][n_out]
void launch_mlp_targets(const DTopo &tp, const MlpDims &md, const double *xt, const double *x, const float *sc,
                        float *Tg, hipStream_t s);
// bfloat16 copies W1b [64][n_in16], W2b [n_out16][64] of the FP32 parameters
void launch_mlp_pack(const MlpDims &md, const float *prm, uint16_t *W1b, uint16_t *W2b, hipStream_t s);
// Z (pre-activations, optional) and Y of the rows of X (rows == null: rows 0..n-1), on the matrix cores
void launch_mlp_forward(int n, const MlpDims &md, const float *X, const int *rows, const float *prm,
                        const uint16_t *W1b, const uint16_t *W2b, float *Z, float *Y, hipStream_t s);
// z = s_F y_F[:dp] on face blocks; cells: mean over their faces of the pressure outputs
template <typename T>
void launch_mlp_scatter(const DTopo &tp, const MlpDims &md, int64_t N, const float *Y, const float *sc, T *z,
                        hipStream_t s);
// gradient g of 1/(2B) sum |Y - T|^2; returns the number of loss partials written
int launch_mlp_backward(int B, int n_in, int n_out, const float *X, const int *rows, const float *Tg,
                        const uint16_t *W2b, const float *Z, const float *Y, float *dY, float *dZ, float *g,
                        double *partial, hipStream_t s);
void launch_mlp_adam(int64_t n, float *prm, const float *g, float *m, float *v, float lr, int step, hipStream_t s);
void launch_mlp_rows(int B, int64_t n, uint64_t seed, int step, int *rows, hipStream_t s);
// minimal residual over {z1, z2 (if m == 2), z3}: x += Z y, r -= W y
template <typename T>
void launch_mr3(int64_t n, int m, const T *z1, const T *z2, const T *z3, const T *w1, const T *w2, const T *w3, T *x,
                T *r, double *partial, double *y, hipStream_t s);
void launch_sum_finish(int G, const double *partial, double *out, hipStream_t s);

// ---- zero-fill ILU of a level operator (natural ordering, structural pattern)
// Rows of one face (group f) or one cell (group n_f + T) share the column list
// gcol[gptr[g], gptr[g+1]) (sorted); row i's values start at LU[voff[i]], its
// diagonal at LU[diag[i]]; L (unit lower) and U share the array.
struct IluDev {
  int64_t N, nface;
  int d, p, t, cond;
  const int64_t *gptr;
  const int32_t *gcol;
  const int64_t *voff, *diag;
  double *LU;
};
// LU = the level operator's values on the pattern
void launch_ilu_fill(const DTopo &tp, const DLevel<double> &L, const IluDev &I, hipStream_t s);
// in-place factorisation, one launch per dependency level (lptr: host prefix of
// the level sizes, lrows: device rows grouped by level); err = row + 1 of a zero pivot
void launch_ilu_factor(const IluDev &I, const int32_t *lrows, const int32_t *lptr, int nlev, int maxrow, int *err,
                       hipStream_t s);
// z = U^{-1} L^{-1} r (forward levels lrows/lptr, backward levels urows/uptr)
void launch_ilu_apply(const IluDev &I, const int32_t *lrows, const int32_t *lptr, int nlevL, const int32_t *urows,
                      const int32_t *uptr, int nlevU, const double *r, double *z, hipStream_t s);

// ---- local HHO operators on the device (one workgroup per cell)
constexpr int kGlTable = 16;       // Gauss-Legendre table stride: n = 1 .. 15 points
constexpr int kLocalThreads = 1024;  // most threads of a cell's workgroup (every rhs_u entry has its own)
struct LocalGeom {
  int d, k, N1, nT, nF, odeg, nf;
  const int32_t *cptr, *cface;  // cell -> faces (the topology's)
  const double *csign;          // [cptr[nc]] +1 if n_F points out of the cell
  const int64_t *fptr, *fvtx;   // face vertices (2D: the two end points)
  const double *verts;          // [nv][d]
  const int64_t *rptr, *ring;   // 2D: counter-clockwise vertex ring of every cell
  const uint8_t *cbox;          // 3D: axis-aligned box cells
  const double *clo, *chi, *apex;
  const double *ccen, *cdiam, *fcen, *fdiam, *fnrm, *ft1, *ft2;
  const int8_t *fbc;
  const double *eta;            // [nc] Nitsche penalty
  const double *glt, *glw;      // [n][kGlTable] nodes and weights on [0, 1]
  const int32_t *EC, *EF;       // exponents of the cell (degree k+1) and face (degree k) monomials
  const double *mf, *fd;        // data against the monomials (see the host's DataMoments)
  const int64_t *foff;
  const int64_t *roff;          // record offsets
  double *rec;                  // records [a | B | rhs_u | rhs_p] (output)
  double *CF;                   // [nf][nF][nF] face bases on the face monomials (formed first)
  int *err;                     // cell + 1 of a degenerate basis or a non-SPD stiffness, -(face + 1)
                                // of a degenerate face basis
};
struct LocalLds {  // LDS layout of the local build (offsets in doubles)
  int C, K, Bc, G, Pi, Nn, gpo, red, rv, gto, scr;
  int max_nq, max_nqf, nloc_max, chunk, threads;
  size_t bytes;
};
LocalLds local_lds(int d, int k, int max_faces, int max_nq, int max_nqf);
void launch_local(const LocalGeom &g, const LocalLds &L, int nc, hipStream_t s);

// ---- batched problems: per-problem (segment) Krylov state over a disjoint union
// A segment's unknowns are its face entries [fo, fo + fl) and cell entries
// [co, co + cl) of the level-0 vector; its "virtual" index e < fl + cl maps to
// fo + e (e < fl) or co + e - fl.
struct SegInfo {
  int64_t fo, fl, co, cl;
};
struct SegChunk {  // kSegChunk consecutive virtual entries of one segment
  int32_t p, e0, len, pad;
};
constexpr int kSegChunk = 4096;
struct GmresState;
void launch_seg_sumsq(int nchunks, const SegChunk *ch, const SegInfo *seg, const double *r, double *partial,
                      hipStream_t s);
// |r_p| -> beta, (bnorm when which == 1), g = beta e1, done flags (sdone[p]);
// which == 2 leaves a segment that is already done untouched
void launch_seg_norm_finish(int np, const int32_t *chunk_ptr, int nchunks, const double *partial, GmresState *st,
                            int *sdone, int which, hipStream_t s);
void launch_seg_scale(int nchunks, const SegChunk *ch, const SegInfo *seg, const double *x, const GmresState *st,
                      double *y, hipStream_t s);
void launch_seg_arnoldi(int mode, int nchunks, const SegChunk *ch, const SegInfo *seg, int np,
                        const int32_t *chunk_ptr, int j, const double *V, int64_t ldv, double *w, double *partial,
                        GmresState *st, int *sdone, int cgs2, hipStream_t s);
void launch_seg_solve_ls(int np, GmresState *st, hipStream_t s);
void launch_seg_combine(int nchunks, const SegChunk *ch, const SegInfo *seg, const double *Z, int64_t ldz,
                        const GmresState *st, double *x, hipStream_t s);
// smoothing step of every segment with its own minimal-residual coefficients
// (y: 3 per segment): x += Z y_p, r -= W y_p over the segment's entries; z3/w3
// null for the two-direction step, m = 1 for one Schwarz direction
template <typename T>
void launch_seg_mr(int nchunks, const SegChunk *ch, const SegInfo *seg, int np, const int32_t *chunk_ptr, int m,
                   const T *z1, const T *z2, const T *z3, const T *w1, const T *w2, const T *w3, T *x, T *r,
                   double *partial, double *y, hipStream_t s);
// *flag = 1 when every sdone[p] is set
void launch_seg_all_done(int np, const int *sdone, int *flag, hipStream_t s);
// v_p -= (v_p . z_p / z_p . z_p) z_p for every segment
void launch_seg_project(int np, const int32_t *chunk_ptr, int nchunks, const SegChunk *ch, const SegInfo *seg,
                        const double *z, double *v, double *partial, double *ratio, hipStream_t s);

// device-resident GMRES scalars
struct GmresState {
  double H[(kMaxRestartH + 1) * kMaxRestartH];
  double h1[kMaxRestartH + 1];
  double h2[kMaxRestartH + 1];
  double cs[kMaxRestartH], sn[kMaxRestartH], g[kMaxRestartH + 1], y[kMaxRestartH];
  double beta;        // norm of the cycle's initial residual
  double bnorm;       // norm of the right-hand side
  double inv_hnext;   // 1 / H[j+1][j]
  double res;         // least-squares residual estimate (absolute)
  double rtol;
  int j;              // current column
  int done;           // converged or broke down
  int nan;            // non-finite value met
  int its;           // Arnoldi steps taken (all cycles)
};

}  // namespace hho
