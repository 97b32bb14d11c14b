// Problem object, device workspace, setup pipeline, V-cycle, coarse solver,
// flexible GMRES, and the C ABI entry points.
#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dev_common.h"
#include "device.h"
#include "internal.h"
#include "k_amg.h"
#include "k_direct.h"
#include "probe.h"

namespace hho {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
void fail(int code, const std::string &msg) { throw Error{code, msg}; }

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess)                                                                           \
      ::hho::fail(HHO_E_DEVICE, std::string("HIP error ") + hipGetErrorString(e_) + " at " #x);    \
  } while (0)

// ------------------------------------------------------------ workspace arena
struct Arena {
  char *base = nullptr;  // null while planning
  size_t off = 0;
  template <typename T>
  T *take(int64_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? (T *)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

template <typename T>
struct VBufs {  // V-cycle vectors of one level
  T *b = nullptr, *w = nullptr, *r = nullptr, *z1 = nullptr, *z2 = nullptr, *w1 = nullptr, *w2 = nullptr,
    *zs0 = nullptr, *zs1 = nullptr;
  T *z3 = nullptr, *w3 = nullptr;  // learned direction (level 0 only)
};

struct LevelInfo {
  int k, p, t, bs;
  int spmv_block = 0, patch_threads = 0;  // autotuned launch shapes (0: defaults)
  int64_t nface, N;
  // FP64 operator and smoother
  double *bsr, *cpl, *spp, *sinv, *xinv, *sig;
  // FP32 copies (mixed V-cycle)
  float *bsr32, *cpl32, *spp32, *sinv32, *xinv32, *sig32;
  // bfloat16 copies of the operator (V-cycle with 16-bit operator storage, FP32 arithmetic)
  bf16 *bsr16, *cpl16, *spp16;
  VBufs<double> v64;
  VBufs<float> v32;
  double *y;  // smoother coefficients
};

// one level's zero-fill ILU (the paper's smoother): the pattern's column list
// per face and per cell, row offsets and diagonals, and the forward (lptr,
// lrows) and backward (uptr, urows) dependency levels
struct IluHost {
  std::vector<int64_t> gptr, voff, diag;
  std::vector<int32_t> gcol, lrows, lptr, urows, uptr;
  int maxrow = 0;
  IluDev dev{};
  int32_t *d_lrows = nullptr, *d_urows = nullptr;
};

// one level's segment table of a batch (the level's vector layout: faces with
// that level's degree, then cells)
struct SegLevel {
  std::vector<SegInfo> hseg;
  std::vector<SegChunk> hch;
  std::vector<int32_t> hptr;
  SegInfo *seg = nullptr;
  SegChunk *ch = nullptr;
  int32_t *ptr = nullptr;
  int G() const { return (int)hch.size(); }
};

}  // namespace hho

using namespace hho;

struct hho_problem {
  const hho_mesh *mesh = nullptr;
  int k = 0, cond = 1, nlev = 1, d = 2;
  std::vector<int> deg;
  hho_options opt;
  double eta = 0;
  LocalData loc;
  bool have_data = false;
  // host topology
  std::vector<int32_t> cptr, cface, fcell, floc, rowptr, col, mirror, blksrc, pairblk;
  std::vector<int64_t> pairoff;
  std::vector<double> zmean;
  int64_t nnzb = 0, ncf = 0;
  int max_faces = 0;
  // device
  char *ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  hipStream_t stream = nullptr;
  bool bound = false, setup_done = false;
  DTopo tp{};
  std::vector<LevelInfo> lev;
  int coarse_dense = 0, border = 0;
  int64_t dense_n = 0;
  // device arrays
  double *rec = nullptr;
  int64_t *roff = nullptr;
  double *stage = nullptr, *rhs_stage = nullptr, *rhs = nullptr, *zvec = nullptr;
  float *stage32 = nullptr;  // V-cycle copy's cell blocks by the matrix-core product (HHO_COPY_PRODUCT)
  double *dense = nullptr, *colbuf = nullptr;
  // outer FGMRES (FP64, level 0) and coarse GMRES (FP64, level L)
  double *oV = nullptr, *oZ = nullptr, *ow = nullptr, *ox = nullptr, *or_ = nullptr, *ob = nullptr;
  double *cV = nullptr, *cZ = nullptr, *cw = nullptr, *cx = nullptr, *cr = nullptr, *czs0 = nullptr,
         *czs1 = nullptr;
  GmresState *ost = nullptr, *cst = nullptr;
  double *partial = nullptr, *scal = nullptr;
  int *err = nullptr;
  // host mirrors
  GmresState *h_st = nullptr;  // pinned
  double timings[16] = {0};
  int64_t coarse_its = 0;  // coarse GMRES iterations of the current solve
  bool uploaded = false;
  // coarsest-level block preconditioner (smoothed aggregation)
  bool coarse_amg = false;
  int amg_nu = 2;
  std::vector<int32_t> fdiag;
  int32_t *d_fdiag = nullptr;
  double *Sd = nullptr;
  AmgHost amgh;
  AmgDev amgd;
  // coarsest-level sparse direct solver (HHO_COARSE_DIRECT)
  bool coarse_direct = false;
  NdHost nd;
  NdDev ndd;
  std::vector<double> zhost;
  size_t lds_condense = 0, lds_patch = 0;
  // batched problems (disjoint union): per-segment FGMRES state
  int nseg = 0;
  std::vector<SegInfo> hseg;
  std::vector<SegChunk> hchunks;
  std::vector<int32_t> hchunk_ptr;
  std::vector<int64_t> seg_face_ptr, seg_cell_ptr;
  std::vector<double> cell_eta;  // per-cell Nitsche penalty of a batch (each member's own default)
  SegInfo *dseg = nullptr;
  SegChunk *dchunks = nullptr;
  int32_t *dchunk_ptr = nullptr;
  GmresState *sst = nullptr;
  int *sdone = nullptr;
  double *seg_partial = nullptr, *seg_ratio = nullptr, *seg_hist = nullptr;
  // per-member scalars inside the V-cycle: segment tables of every level, the
  // smoothing steps' coefficients (3 per member) and the coarse GMRES state
  std::vector<SegLevel> segl;
  double *seg_y = nullptr;
  GmresState *csst = nullptr;
  int *csdone = nullptr, *call_done = nullptr;
  std::vector<int> seg_its;
  std::vector<std::vector<double>> seg_hist_h;  // per-member residual estimates of the last batched solve
  bool opt_seg_hist = false;                     // record them (hho_batch_solve with histories)
  std::vector<double> seg_rel;
  // the paper's smoother: zero-fill ILU per level (options.smoother = ILU)
  bool ilu_on = false;
  std::vector<IluHost> ilu;  // per level; empty pattern where the level takes none
  // the V-cycle as a replayed HIP graph (hho_set_graph)
  bool graph_on = false, in_capture = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int64_t gkey = -1;
  hipStream_t cap_stream = nullptr;  // captures (the caller's stream may be the legacy one)
  // local operators built on the device (options.local_build)
  bool local_dev = false;
  DataMoments dmom;
  LocalGeomHost lgeo;
  LocalLds llds{};
  LocalGeom lg{};
  double *d_user_rhs = nullptr;          // hho_set_moments with the device build: [rhs_u | rhs_p] per cell
  int64_t *d_user_off = nullptr;         // [nc+1] offsets of those packed records
  std::vector<double> user_rhs;          // empty: the device build's own right-hand side
  std::vector<int64_t> user_off;
  std::vector<double> cell_eta_dev;      // penalty of every cell for the device build
  // learned fine-level smoother
  MlpDims md{};
  bool learned_on = false, learned_ready = false;
  int adam_step = 0;
  uint16_t *mlp_w1b = nullptr, *mlp_w2b = nullptr;  // bfloat16 copies of the weights
  float *mlp_prm = nullptr, *mlp_g = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_X = nullptr, *mlp_sc = nullptr,
        *mlp_Y = nullptr, *mlp_Z = nullptr, *mlp_dZ = nullptr, *mlp_Yb = nullptr, *mlp_dY = nullptr;
  int *mlp_rows = nullptr;
  double *mlp_loss = nullptr;
  // live timing of armed kernel classes (hho_probe_arm / hho_probe_read)
  KernelProbe probe;
};

namespace hho {

static int level_t(const hho_problem *P, int k) { return P->cond == HHO_COND_V ? dim_poly(P->d, k) : 1; }

// Every device array of the problem, in one place: run once to size the
// workspace (base == null) and once to hand out pointers.
// The level takes the ILU smoother: every smoothed level, and the coarsest
// when its solve is GMRES preconditioned by the smoother's preconditioner.
static bool ilu_level(const hho_problem *P, int l) {
  if (!P->ilu_on) return false;
  const int Lc = P->nlev - 1;
  return l < Lc || (!P->coarse_dense && !P->coarse_amg && !P->coarse_direct);
}

// Pattern of the level operator in the natural ordering: a face's rows share
// the unknowns of its (at most two) cells, a cell's rows its own unknowns.
static void build_ilu_level(hho_problem *P, int l, IluHost &H) {
  const LevelInfo &L = P->lev[l];
  const int d = P->d, p = L.p, t = L.t, dp = d * p;
  const int64_t nf = P->mesh->nf, nc = P->mesh->nc, nface = L.nface, N = L.N;
  if (N >= INT32_MAX) fail(HHO_E_INVALID_ARG, "ILU smoother: level too large");
  H = IluHost{};
  H.gptr.assign(1, 0);
  std::vector<int32_t> faces;
  std::vector<int32_t> cells;
  auto emit = [&]() {
    std::sort(faces.begin(), faces.end());
    faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
    std::sort(cells.begin(), cells.end());
    for (int32_t g : faces)
      for (int r = 0; r < dp; ++r) H.gcol.push_back((int32_t)((int64_t)g * dp + r));
    for (int32_t T : cells)
      for (int q = 0; q < t; ++q) H.gcol.push_back((int32_t)(nface + (int64_t)T * t + q));
    H.gptr.push_back((int64_t)H.gcol.size());
  };
  for (int64_t f = 0; f < nf; ++f) {
    faces.clear();
    cells.clear();
    for (int sd = 0; sd < 2; ++sd) {
      const int T = P->fcell[2 * f + sd];
      if (T < 0) continue;
      cells.push_back(T);
      for (int e = P->cptr[T]; e < P->cptr[T + 1]; ++e) faces.push_back(P->cface[e]);
    }
    emit();
  }
  for (int64_t T = 0; T < nc; ++T) {
    faces.assign(P->cface.begin() + P->cptr[T], P->cface.begin() + P->cptr[T + 1]);
    cells.assign(1, (int32_t)T);
    emit();
  }
  auto group = [&](int64_t i) { return i < nface ? i / dp : nf + (i - nface) / t; };
  H.voff.assign(N + 1, 0);
  H.diag.assign(N, 0);
  for (int64_t i = 0; i < N; ++i) {
    const int64_t g = group(i), b = H.gptr[g], len = H.gptr[g + 1] - b;
    H.maxrow = std::max<int>(H.maxrow, (int)len);
    H.voff[i + 1] = H.voff[i] + len;
    const int32_t *c = H.gcol.data() + b;
    const int64_t pos = std::lower_bound(c, c + len, (int32_t)i) - c;
    if (pos >= len || c[pos] != i) fail(HHO_E_INVALID_ARG, "ILU smoother: row without its diagonal");
    H.diag[i] = H.voff[i] + pos;
  }
  // dependency levels: forward over the columns left of the diagonal, backward right of it
  std::vector<int32_t> lf(N, 0), lb(N, 0);
  int nlf = 0, nlb = 0;
  for (int64_t i = 0; i < N; ++i) {
    const int64_t g = group(i), b = H.gptr[g];
    const int64_t dl = H.diag[i] - H.voff[i];
    int m = 0;
    for (int64_t e = 0; e < dl; ++e) m = std::max(m, lf[H.gcol[b + e]]);
    lf[i] = m + 1;
    nlf = std::max(nlf, m + 1);
  }
  for (int64_t i = N - 1; i >= 0; --i) {
    const int64_t g = group(i), b = H.gptr[g], len = H.gptr[g + 1] - b;
    const int64_t dl = H.diag[i] - H.voff[i];
    int m = 0;
    for (int64_t e = dl + 1; e < len; ++e) m = std::max(m, lb[H.gcol[b + e]]);
    lb[i] = m + 1;
    nlb = std::max(nlb, m + 1);
  }
  auto bucket = [&](const std::vector<int32_t> &lv, int nl, std::vector<int32_t> &ptr, std::vector<int32_t> &rows) {
    ptr.assign(nl + 1, 0);
    for (int64_t i = 0; i < N; ++i) ++ptr[lv[i]];
    for (int k = 0; k < nl; ++k) ptr[k + 1] += ptr[k];  // level k + 1 (1-based) holds rows [ptr[k], ptr[k+1])
    rows.assign(N, 0);
    std::vector<int32_t> at(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < N; ++i) rows[at[lv[i] - 1]++] = (int32_t)i;
  };
  bucket(lf, nlf, H.lptr, H.lrows);
  bucket(lb, nlb, H.uptr, H.urows);
  if (H.maxrow * 4 * (int64_t)sizeof(double) > (int64_t)kMaxLdsBytes - 1024)
    fail(HHO_E_INVALID_ARG, "ILU smoother: a row of the pattern exceeds the LDS staging");
  H.dev.N = N;
  H.dev.nface = nface;
  H.dev.d = d;
  H.dev.p = p;
  H.dev.t = t;
  H.dev.cond = P->cond;
}

static void plan(hho_problem *P, Arena &A) {
  const int d = P->d;
  const int64_t nc = P->mesh->nc, nf = P->mesh->nf;
  // levels above the coarsest run in FP32 arithmetic (FP32 or bfloat16 storage)
  const bool mixed = P->opt.precision != HHO_PREC_FP64;
  const bool b16 = P->opt.precision == HHO_PREC_BF16;
  // topology
  P->tp.cptr = A.take<int32_t>(nc + 1);
  P->tp.cface = A.take<int32_t>(P->ncf);
  P->tp.fcell = A.take<int32_t>(2 * nf);
  P->tp.floc = A.take<int32_t>(2 * nf);
  P->tp.rowptr = A.take<int32_t>(nf + 1);
  P->tp.col = A.take<int32_t>(P->nnzb);
  P->tp.mirror = A.take<int32_t>(P->nnzb);
  P->tp.blksrc = A.take<int32_t>(6 * P->nnzb);
  P->tp.pairoff = A.take<int64_t>(nc + 1);
  P->tp.pairblk = A.take<int32_t>(P->pairoff[nc]);
  P->tp.zmean = A.take<double>(nc);
  // local records and condensation staging
  P->rec = A.take<double>(P->loc.off.empty() ? 1 : P->loc.off[nc]);
  P->roff = A.take<int64_t>(nc + 1);
  if (P->local_dev) {
    const hho_mesh *m = P->mesh;
    LocalGeom &g = P->lg;
    g.d = d;
    g.k = P->k;
    g.N1 = P->loc.N1;
    g.nT = P->loc.nT;
    g.nF = P->loc.nF;
    g.odeg = P->lgeo.odeg;
    g.nf = (int)P->mesh->nf;
    g.cptr = P->tp.cptr;
    g.cface = P->tp.cface;
    g.csign = A.take<double>(m->csign.size());
    g.fptr = A.take<int64_t>(m->fptr.size());
    g.fvtx = A.take<int64_t>(m->fvtx.size());
    g.verts = A.take<double>(m->verts.size());
    g.rptr = A.take<int64_t>(P->lgeo.rptr.size());
    g.ring = A.take<int64_t>(std::max<size_t>(1, P->lgeo.ring.size()));
    g.cbox = A.take<uint8_t>(std::max<size_t>(1, m->cbox.size()));
    g.clo = A.take<double>(std::max<size_t>(1, m->clo.size()));
    g.chi = A.take<double>(std::max<size_t>(1, m->chi.size()));
    g.apex = A.take<double>(P->lgeo.apex.size());
    g.ccen = A.take<double>(m->ccen.size());
    g.cdiam = A.take<double>(m->cdiam.size());
    g.fcen = A.take<double>(m->fcen.size());
    g.fdiam = A.take<double>(m->fdiam.size());
    g.fnrm = A.take<double>(m->fnrm.size());
    g.ft1 = A.take<double>(m->ft1.size());
    g.ft2 = A.take<double>(m->ft2.size());
    g.fbc = A.take<int8_t>(m->fbc.size());
    g.eta = A.take<double>(nc);
    g.glt = A.take<double>(P->lgeo.glt.size());
    g.glw = A.take<double>(P->lgeo.glw.size());
    g.EC = A.take<int32_t>(P->lgeo.EC.size());
    g.EF = A.take<int32_t>(std::max<size_t>(1, P->lgeo.EF.size()));
    g.mf = A.take<double>(std::max<size_t>(1, P->dmom.mf.size()));
    g.fd = A.take<double>(std::max<size_t>(1, P->dmom.fd.size()));
    g.foff = A.take<int64_t>(P->dmom.foff.size());
    g.roff = P->roff;
    g.rec = P->rec;
    g.err = nullptr;  // set below, once the error slots are placed
    int64_t nu = 0;
    for (int32_t v : P->loc.nloc) nu += (int64_t)d * v + P->loc.nT;
    g.CF = A.take<double>(std::max<int64_t>(1, (int64_t)P->mesh->nf * g.nF * g.nF));
    P->d_user_rhs = A.take<double>(std::max<int64_t>(1, nu));
    P->d_user_off = A.take<int64_t>(nc + 1);
  }
  const LevelInfo &L0 = P->lev[0];
  P->stage = A.take<double>(P->pairoff[nc] * L0.bs * L0.bs);
  P->stage32 = P->opt.vcycle_copy == HHO_COPY_PRODUCT ? A.take<float>(P->pairoff[nc] * L0.bs * L0.bs) : nullptr;
  P->rhs_stage = A.take<double>(P->ncf * d * L0.p);
  P->rhs = A.take<double>(L0.N);
  P->zvec = A.take<double>(L0.N);
  const int Lc = P->nlev - 1;
  for (int l = 0; l < P->nlev; ++l) {
    LevelInfo &L = P->lev[l];
    const int64_t nbsr = P->nnzb * L.bs * L.bs;
    const int64_t ncpl = P->ncf * d * L.p * (P->cond == HHO_COND_V ? L.t : 1);
    const int64_t nspp = P->cond == HHO_COND_V ? nc * L.t * L.t : 1;
    const int64_t nsinv = P->pairoff[nc] * L.bs * L.bs;
    const int64_t nxinv = P->cond == HHO_COND_V ? nc * L.t * L.t : P->ncf * d * L.p;
    L.bsr = A.take<double>(nbsr);
    L.cpl = A.take<double>(ncpl);
    L.spp = A.take<double>(nspp);
    const bool need_smoother = (l < Lc) || !(P->coarse_dense || P->coarse_direct);
    L.sinv = need_smoother ? A.take<double>(nsinv) : nullptr;
    L.xinv = need_smoother ? A.take<double>(nxinv) : nullptr;
    L.sig = need_smoother ? A.take<double>(nc) : nullptr;
    L.y = A.take<double>(4);
    if (mixed && l < Lc) {
      // bfloat16 mode: operator values in 16 bits; the smoother's factors stay FP32
      // (its packed-row loads are bound by their count, not their width)
      if (b16) {
        L.bsr16 = A.take<bf16>(nbsr);
        L.cpl16 = A.take<bf16>(ncpl);
        L.spp16 = A.take<bf16>(nspp);
      } else {
        L.bsr32 = A.take<float>(nbsr);
        L.cpl32 = A.take<float>(ncpl);
        L.spp32 = A.take<float>(nspp);
      }
      L.sinv32 = A.take<float>(nsinv);
      L.xinv32 = A.take<float>(nxinv);
      L.sig32 = A.take<float>(nc);
    }
    auto vecs = [&](auto &V, auto tag) {
      using T = decltype(tag);
      V.b = A.take<T>(L.N);
      V.w = A.take<T>(L.N);
      V.r = A.take<T>(L.N);
      V.z1 = A.take<T>(L.N);
      V.z2 = A.take<T>(L.N);
      V.w1 = A.take<T>(L.N);
      V.w2 = A.take<T>(L.N);
      V.zs0 = A.take<T>(L.N);
      V.zs1 = A.take<T>(L.nface);
      if (P->opt.learned && l == 0) {
        V.z3 = A.take<T>(L.N);
        V.w3 = A.take<T>(L.N);
      }
    };
    if (l == Lc || !mixed)
      vecs(L.v64, 0.0);
    else
      vecs(L.v32, 0.0f);
  }
  // coarse solver
  const LevelInfo &LC = P->lev[Lc];
  if (P->coarse_dense) {
    P->dense = A.take<double>(P->dense_n * 2 * P->dense_n);
    P->colbuf = A.take<double>(P->dense_n);
  } else if (P->coarse_direct) {
    NdHost &H = P->nd;
    if (H.m.empty())
      nd_symbolic(P->mesh, d, LC.p, LC.t, P->cond, P->border != 0, P->rowptr, P->col, P->seg_cell_ptr, &H);
    if ((int64_t)H.maxm * (int64_t)sizeof(double) > (int64_t)kMaxLdsBytes - 1024)
      fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: a front exceeds the LDS of one compute unit");
    NdDev &D = P->ndd;
    const int nn = H.nfront;
    D.m = A.take<int32_t>(nn);
    D.nfs = A.take<int32_t>(nn);
    D.child = A.take<int32_t>(2 * nn);
    D.off = A.take<int64_t>(nn + 1);
    D.voff = A.take<int64_t>(nn + 1);
    D.dofoff = A.take<int64_t>(nn + 1);
    D.soff = A.take<int64_t>(nn);
    D.dof = A.take<int32_t>(H.dof.size());
    D.cmap = A.take<int32_t>(H.cmap.size());
    D.npair = (int64_t)H.src.size();
    D.src = A.take<int64_t>(H.src.size());
    D.dst = A.take<int64_t>(H.dst.size());
    D.hfront = A.take<int32_t>(H.hfront.size());
    D.tiles = A.take<int32_t>(H.tiles.size());
    D.chunks = A.take<int32_t>(H.chunks.size());
    D.schunks = A.take<int32_t>(H.schunks.size());
    D.F = A.take<double>(H.total);
    D.V = A.take<double>(H.vtotal);
    D.S = A.take<double>(H.stotal);
    D.coef = A.take<double>(H.pins.size());
    D.pins = A.take<int64_t>(H.pins.size());
    D.segp = A.take<int64_t>(H.segp.size());
    D.cseg = A.take<int32_t>(H.cseg.size());
  } else {
    const int R = P->opt.coarse_restart;
    P->cV = A.take<double>((int64_t)(R + 1) * LC.N);
    P->cZ = A.take<double>((int64_t)R * LC.N);
    P->cw = A.take<double>(LC.N);
    P->cr = A.take<double>(LC.N);
    P->czs0 = A.take<double>(LC.N);
    P->czs1 = A.take<double>(LC.nface);
  }
  // smoothed-aggregation hierarchy of the coarsest level
  if (P->coarse_amg) {
    P->d_fdiag = A.take<int32_t>(nf);
    P->Sd = A.take<double>(nc);
    AmgDev &D = P->amgd;
    D.probe = &P->probe;
    D.nlev = (int)P->amgh.levels.size();
    for (int l = 0; l < D.nlev; ++l) {
      const AmgHostLevel &H = P->amgh.levels[l];
      AmgDevLevel &G = D.lev[l];
      G.n = H.n;
      G.nc = H.nc;
      G.nnz = (int64_t)H.ci.size();
      G.npe = (int64_t)H.pci.size();
      G.nbe = (int64_t)H.bci.size();
      G.rp = A.take<int32_t>(H.rp.size());
      G.ci = A.take<int32_t>(H.ci.size());
      G.diag = A.take<int32_t>(H.diag.size());
      G.val = A.take<double>(G.nnz);
      G.dinv = A.take<double>(G.n);
      G.lam = A.take<double>(1);
      G.x = A.take<double>((int64_t)G.n * d);
      G.r = A.take<double>((int64_t)G.n * d);
      G.res = A.take<double>((int64_t)G.n * d);
      G.tmp = A.take<double>((int64_t)G.n * d);
      if (H.nc > 0) {
        G.prp = A.take<int32_t>(H.prp.size());
        G.pci = A.take<int32_t>(H.pci.size());
        G.prow = A.take<int32_t>(H.pci.size());
        G.pgp = A.take<int32_t>(H.pgp.size());
        G.pgi = A.take<int32_t>(H.pgi.size());
        G.pself = A.take<int32_t>(H.pself.size());
        G.pval = A.take<double>(G.npe);
        G.np1 = H.np1;
        if (H.np1 > 0) {
          G.p1row = A.take<int32_t>(H.p1row.size());
          G.qpp = A.take<int32_t>(H.qpp.size());
          G.qpa = A.take<int32_t>(H.qpa.size());
          G.qpb = A.take<int32_t>(H.qpb.size());
          G.p2src = A.take<int32_t>(H.p2src.size());
          G.pval1 = A.take<double>(H.np1);
          G.qval = A.take<double>(G.npe);
        }
        G.ptp = A.take<int32_t>(H.ptp.size());
        G.pti = A.take<int32_t>(H.pti.size());
        G.pte = A.take<int32_t>(H.pte.size());
        G.bpp = A.take<int32_t>(H.bpp.size());
        G.bpa = A.take<int32_t>(H.bpa.size());
        G.bpb = A.take<int32_t>(H.bpb.size());
        G.brp = A.take<int32_t>(H.brp.size());
        G.bci = A.take<int32_t>(H.bci.size());
        G.btp = A.take<int32_t>(H.btp.size());
        G.bti = A.take<int32_t>(H.bti.size());
        G.bte = A.take<int32_t>(H.bte.size());
        G.bval = A.take<double>(G.nbe);
        G.ptval = A.take<double>(G.npe);
        G.btval = A.take<double>(G.nbe);
        G.cpp = A.take<int32_t>(H.cpp.size());
        G.cpa = A.take<int32_t>(H.cpa.size());
        G.cpb = A.take<int32_t>(H.cpb.size());
      }
    }
    // explicit V-cycle operator from the first level with at most
    // coarse_amg_explicit rows down (none if that is the dense coarsest level)
    D.expl = -1;
    for (int l = 0; l < D.nlev; ++l)
      if (D.lev[l].n <= P->opt.coarse_amg_explicit) {
        if (!(l == D.nlev - 1 && D.lev[l].n <= kAmgCoarsest)) D.expl = l;
        break;
      }
    if (D.expl >= 0) {
      const int64_t m = D.lev[D.expl].n;
      for (int l = D.expl; l < D.nlev; ++l) {
        D.cr[l] = A.take<double>(D.lev[l].n * m);
        D.cx[l] = A.take<double>(D.lev[l].n * m);
        D.ct[l] = A.take<double>(D.lev[l].n * m);
      }
      D.mexpl = D.cx[D.expl];
    }
    const int nlast = P->amgh.levels.back().n;
    if (nlast <= kAmgCoarsest) {  // dense inverse of the coarsest level; Jacobi sweeps above that size
      D.ainv = A.take<double>((int64_t)nlast * nlast);
      D.dense_scratch = A.take<double>((int64_t)nlast * nlast);
    } else {
      D.ainv = D.dense_scratch = nullptr;
    }
    D.partial = A.take<double>(512);
  }
  // batched problems
  if (P->nseg > 0) {
    const int64_t G = (int64_t)P->hchunks.size();
    P->dseg = A.take<SegInfo>(P->nseg);
    P->dchunks = A.take<SegChunk>(G);
    P->dchunk_ptr = A.take<int32_t>(P->nseg + 1);
    P->sst = A.take<GmresState>(P->nseg);
    P->sdone = A.take<int>(P->nseg);
    P->seg_partial = A.take<double>(G * (kMaxRestartH + 2));
    P->seg_ratio = A.take<double>(P->nseg);
    P->seg_hist = A.take<double>(2 * P->nseg);
    for (int l = 0; l < P->nlev; ++l) {
      SegLevel &S = P->segl[l];
      if (l == 0) {
        S.seg = P->dseg;
        S.ch = P->dchunks;
        S.ptr = P->dchunk_ptr;
      } else {
        S.seg = A.take<SegInfo>(P->nseg);
        S.ch = A.take<SegChunk>(S.G());
        S.ptr = A.take<int32_t>(P->nseg + 1);
      }
    }
    P->seg_y = A.take<double>(3 * P->nseg);
    P->csst = A.take<GmresState>(P->nseg);
    P->csdone = A.take<int>(P->nseg);
    P->call_done = A.take<int>(1);
  }
  // the paper's smoother: ILU patterns (built once) and factors
  if (P->ilu_on) {
    if (P->ilu.size() != (size_t)P->nlev) P->ilu.assign(P->nlev, IluHost{});
    for (int l = 0; l < P->nlev; ++l) {
      if (!ilu_level(P, l)) continue;
      IluHost &H = P->ilu[l];
      if (H.gptr.empty()) build_ilu_level(P, l, H);
      const int64_t N = P->lev[l].N;
      H.dev.gptr = A.take<int64_t>(H.gptr.size());
      H.dev.gcol = A.take<int32_t>(H.gcol.size());
      H.dev.voff = A.take<int64_t>(N + 1);
      H.dev.diag = A.take<int64_t>(N);
      H.dev.LU = A.take<double>(H.voff[N]);
      H.d_lrows = A.take<int32_t>(N);
      H.d_urows = A.take<int32_t>(N);
    }
  }
  // learned fine-level smoother
  if (P->opt.learned) {
    const MlpDims &md = P->md;
    const int64_t np = mlp_param_count(md);
    P->mlp_prm = A.take<float>(np);
    P->mlp_w1b = A.take<uint16_t>((int64_t)kMlpHidden * md.n_in16);
    P->mlp_w2b = A.take<uint16_t>((int64_t)md.n_out16 * kMlpHidden);
    P->mlp_g = A.take<float>(np);
    P->mlp_m = A.take<float>(np);
    P->mlp_v = A.take<float>(np);
    P->mlp_X = A.take<float>(nf * (int64_t)md.n_in);
    P->mlp_sc = A.take<float>(nf);
    P->mlp_Y = A.take<float>(nf * (int64_t)md.n_out);
    P->mlp_rows = A.take<int>(kMlpMaxBatch);
    P->mlp_Z = A.take<float>((int64_t)kMlpMaxBatch * kMlpHidden);
    P->mlp_dZ = A.take<float>((int64_t)kMlpMaxBatch * kMlpHidden);
    P->mlp_Yb = A.take<float>((int64_t)kMlpMaxBatch * md.n_out);
    P->mlp_dY = A.take<float>((int64_t)kMlpMaxBatch * md.n_out);
    P->mlp_loss = A.take<double>(kMlpMaxSteps);
  }
  // outer FGMRES
  const int R = P->opt.restart;
  P->oV = A.take<double>((int64_t)(R + 1) * L0.N);
  P->oZ = A.take<double>((int64_t)R * L0.N);
  P->ow = A.take<double>(L0.N);
  P->ox = A.take<double>(L0.N);
  P->or_ = A.take<double>(L0.N);
  P->ob = A.take<double>(L0.N);
  P->ost = A.take<GmresState>(1);
  P->cst = A.take<GmresState>(1);
  P->partial = A.take<double>(512 * (kMaxRestartH + 2));
  P->scal = A.take<double>(16);
  P->err = A.take<int>(8);
  if (P->local_dev) P->lg.err = P->err + 4;
}

static DLevel<double> dlev64(const hho_problem *P, int l) {
  const LevelInfo &L = P->lev[l];
  DLevel<double> D;
  D.cond = P->cond;
  D.p = L.p;
  D.t = L.t;
  D.nface = L.nface;
  D.N = L.N;
  D.bsr = L.bsr;
  D.cpl = L.cpl;
  D.spp = L.spp;
  D.sinv = L.sinv;
  D.xinv = L.xinv;
  D.sig = L.sig;
  D.block = L.spmv_block;
  return D;
}
static DLevel<float> dlev32(const hho_problem *P, int l) {
  const LevelInfo &L = P->lev[l];
  DLevel<float> D;
  D.cond = P->cond;
  D.p = L.p;
  D.t = L.t;
  D.nface = L.nface;
  D.N = L.N;
  D.bsr = L.bsr32;
  D.cpl = L.cpl32;
  D.spp = L.spp32;
  D.sinv = L.sinv32;
  D.xinv = L.xinv32;
  D.sig = L.sig32;
  D.block = L.spmv_block;
  return D;
}
static DLevel<float, bf16, float> dlev16(const hho_problem *P, int l) {
  const LevelInfo &L = P->lev[l];
  DLevel<float, bf16, float> D;
  D.cond = P->cond;
  D.p = L.p;
  D.t = L.t;
  D.nface = L.nface;
  D.N = L.N;
  D.bsr = L.bsr16;
  D.cpl = L.cpl16;
  D.spp = L.spp16;
  D.sinv = L.sinv32;
  D.xinv = L.xinv32;
  D.sig = L.sig32;
  D.block = L.spmv_block;
  return D;
}
// V-cycle precisions: vector/arithmetic type T and value storage Sto
struct PrecF64 {
  using T = double;
  static DLevel<double> op(const hho_problem *P, int l) { return dlev64(P, l); }
  static VBufs<double> &vb(hho_problem *P, int l) { return P->lev[l].v64; }
};
struct PrecF32 {
  using T = float;
  static DLevel<float> op(const hho_problem *P, int l) { return dlev32(P, l); }
  static VBufs<float> &vb(hho_problem *P, int l) { return P->lev[l].v32; }
};
struct PrecB16 {
  using T = float;
  static DLevel<float, bf16, float> op(const hho_problem *P, int l) { return dlev16(P, l); }
  static VBufs<float> &vb(hho_problem *P, int l) { return P->lev[l].v32; }
};

static void build_topology(hho_problem *P) {
  const hho_mesh *m = P->mesh;
  const int64_t nc = m->nc, nf = m->nf;
  if (m->cface.size() > (size_t)INT32_MAX || nf > INT32_MAX || nc > INT32_MAX)
    fail(HHO_E_INVALID_ARG, "mesh too large for 32-bit indices");
  P->ncf = (int64_t)m->cface.size();
  P->cptr.assign(m->cptr.begin(), m->cptr.end());
  P->cface.assign(m->cface.begin(), m->cface.end());
  P->fcell.resize(2 * nf);
  P->floc.resize(2 * nf);
  for (int64_t f = 0; f < nf; ++f)
    for (int s = 0; s < 2; ++s) {
      P->fcell[2 * f + s] = (int32_t)m->fcell[s][f];
      P->floc[2 * f + s] = m->flocal[s][f];
    }
  // face-block rows: faces of the cells sharing the face
  P->rowptr.assign(nf + 1, 0);
  std::vector<std::vector<int32_t>> nb(nf);
  for (int64_t f = 0; f < nf; ++f) {
    for (int s = 0; s < 2; ++s) {
      int64_t c = m->fcell[s][f];
      if (c < 0) continue;
      for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e) nb[f].push_back((int32_t)m->cface[e]);
    }
    std::sort(nb[f].begin(), nb[f].end());
    nb[f].erase(std::unique(nb[f].begin(), nb[f].end()), nb[f].end());
    P->rowptr[f + 1] = P->rowptr[f] + (int32_t)nb[f].size();
  }
  P->nnzb = P->rowptr[nf];
  P->col.resize(P->nnzb);
  for (int64_t f = 0; f < nf; ++f) std::copy(nb[f].begin(), nb[f].end(), P->col.begin() + P->rowptr[f]);
  P->blksrc.assign(6 * P->nnzb, -1);
  P->pairoff.assign(nc + 1, 0);
  for (int64_t c = 0; c < nc; ++c) {
    int64_t n = m->cptr[c + 1] - m->cptr[c];
    P->pairoff[c + 1] = P->pairoff[c] + n * n;
  }
  P->pairblk.assign(P->pairoff[nc], -1);
  for (int64_t c = 0; c < nc; ++c) {
    int n = (int)(m->cptr[c + 1] - m->cptr[c]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        int32_t fi = (int32_t)m->cface[m->cptr[c] + i], fj = (int32_t)m->cface[m->cptr[c] + j];
        auto b0 = P->col.begin() + P->rowptr[fi], b1 = P->col.begin() + P->rowptr[fi + 1];
        auto it = std::lower_bound(b0, b1, fj);
        int64_t b = it - P->col.begin();
        P->pairblk[P->pairoff[c] + i * n + j] = (int32_t)b;
        int s = P->blksrc[6 * b] < 0 ? 0 : 1;
        if (s == 1 && P->blksrc[6 * b + 3] >= 0) fail(HHO_E_MESH, "face block with more than two cells");
        P->blksrc[6 * b + 3 * s] = (int32_t)c;
        P->blksrc[6 * b + 3 * s + 1] = i;
        P->blksrc[6 * b + 3 * s + 2] = j;
      }
  }
  // mirror block: (f, g) -> (g, f); the operator is symmetric, so the transpose of
  // the mirror block is the block itself (column access becomes contiguous)
  P->mirror.assign(P->nnzb, -1);
  for (int64_t f = 0; f < nf; ++f)
    for (int32_t b = P->rowptr[f]; b < P->rowptr[f + 1]; ++b) {
      const int32_t g = P->col[b];
      auto b0 = P->col.begin() + P->rowptr[g], b1 = P->col.begin() + P->rowptr[g + 1];
      auto it = std::lower_bound(b0, b1, (int32_t)f);
      if (it == b1 || *it != (int32_t)f) fail(HHO_E_MESH, "face-block pattern is not symmetric");
      P->mirror[b] = (int32_t)(it - P->col.begin());
    }
  P->fdiag.assign(nf, -1);
  for (int64_t f = 0; f < nf; ++f) {
    auto b0 = P->col.begin() + P->rowptr[f], b1 = P->col.begin() + P->rowptr[f + 1];
    P->fdiag[f] = (int32_t)(std::lower_bound(b0, b1, (int32_t)f) - P->col.begin());
  }
  P->zmean.resize(nc);
  for (int64_t c = 0; c < nc; ++c) P->zmean[c] = std::sqrt(m->cvol[c]);
  P->max_faces = m->max_faces;
  P->tp.d = P->d;
  P->tp.max_faces = m->max_faces;
  P->tp.nc = (int)nc;
  P->tp.nf = (int)nf;
  P->tp.ncf = P->ncf;
  P->tp.nnzb = P->nnzb;
}

static void init_levels(hho_problem *P) {
  P->lev.resize(P->nlev);
  for (int l = 0; l < P->nlev; ++l) {
    LevelInfo &L = P->lev[l];
    L = LevelInfo{};
    L.k = P->deg[l];
    L.p = dim_poly(P->d - 1, L.k);
    L.t = level_t(P, L.k);
    L.bs = P->cond == HHO_COND_V ? L.p : P->d * L.p;
    L.nface = P->mesh->nf * P->d * L.p;
    L.N = L.nface + P->mesh->nc * L.t;
  }
  const LevelInfo &LC = P->lev[P->nlev - 1];
  P->border = (P->mesh->has_neumann || P->opt.nullspace == HHO_NULLSPACE_NONE) ? 0 : 1;
  const int64_t nd = LC.N + P->border;
  P->coarse_dense = (P->opt.coarse_mode == HHO_COARSE_DENSE) ||
                    (P->opt.coarse_mode == HHO_COARSE_AUTO && nd <= 1024 && !(P->nseg > 1 && P->border));
  if (P->coarse_dense && P->nseg > 1 && P->border)
    fail(HHO_E_INVALID_ARG, "a batch of problems with pure Dirichlet boundaries needs an iterative coarse solver");
  if (P->coarse_dense && nd > 8192) fail(HHO_E_INVALID_ARG, "dense coarse solver limited to 8192 unknowns");
  P->dense_n = nd;
  P->coarse_direct = !P->coarse_dense && (P->opt.coarse_mode == HHO_COARSE_DIRECT ||
                                          (P->opt.coarse_mode == HHO_COARSE_AUTO && LC.k == 0));
  if (P->coarse_direct && LC.k != 0) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver needs a coarsest degree of 0");
  P->nd = NdHost{};  // built when the workspace is planned
  P->coarse_amg = !P->coarse_dense && !P->coarse_direct &&
                  (P->opt.coarse_mode == HHO_COARSE_AMG || (P->opt.coarse_mode == HHO_COARSE_AUTO && LC.k == 0));
  if (P->coarse_amg && LC.k != 0) fail(HHO_E_INVALID_ARG, "AMG coarse solver needs a coarsest degree of 0");
  P->amgh.levels.clear();  // built by amg_levels() once the problem's data are set
}

// AUTO's sparse direct solve only while its fronts fit: their storage within
// kNdAutoBytes and the largest front within the solve kernels' LDS; otherwise
// the AMG-preconditioned GMRES (decided once the symbolic phase has run)
constexpr int64_t kNdAutoBytes = int64_t(32) << 30;
static void settle_auto_coarse(hho_problem *P) {
  if (P->opt.coarse_mode != HHO_COARSE_AUTO || !P->coarse_direct || !P->nd.m.empty()) return;
  const LevelInfo &LC = P->lev[P->nlev - 1];
  nd_symbolic(P->mesh, P->d, LC.p, LC.t, P->cond, P->border != 0, P->rowptr, P->col, P->seg_cell_ptr, &P->nd);
  const NdHost &H = P->nd;
  if (H.total * (int64_t)sizeof(double) <= kNdAutoBytes &&
      (int64_t)H.maxm * (int64_t)sizeof(double) <= (int64_t)kMaxLdsBytes - 1024)
    return;
  P->nd = NdHost{};
  P->coarse_direct = false;
  P->coarse_amg = true;
}

// symbolic smoothed-aggregation hierarchy of the coarsest level (topology only)
static void amg_levels(hho_problem *P) {
  if (!P->coarse_amg || !P->amgh.levels.empty()) return;
  amg_symbolic((int)P->mesh->nf, P->rowptr.data(), P->col.data(), kAmgCoarsest, P->opt.coarse_amg_psmooth,
               &P->amgh);
  if ((int)P->amgh.levels.size() > kMaxAmgLevels) fail(HHO_E_INVALID_ARG, "AMG hierarchy too deep");
}

static void check_device_error(hho_problem *P, const char *what) {
  HIPCHK(hipGetLastError());
  (void)P;
  (void)what;
}

// ------------------------------------------------------------ setup
static void device_upload(hho_problem *P) {
  hipStream_t s = P->stream;
  auto h2d = [&](void *dst, const void *src, size_t bytes) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
  };
  h2d((void *)P->tp.cptr, P->cptr.data(), P->cptr.size() * 4);
  h2d((void *)P->tp.cface, P->cface.data(), P->cface.size() * 4);
  h2d((void *)P->tp.fcell, P->fcell.data(), P->fcell.size() * 4);
  h2d((void *)P->tp.floc, P->floc.data(), P->floc.size() * 4);
  h2d((void *)P->tp.rowptr, P->rowptr.data(), P->rowptr.size() * 4);
  h2d((void *)P->tp.col, P->col.data(), P->col.size() * 4);
  h2d((void *)P->tp.mirror, P->mirror.data(), P->mirror.size() * 4);
  h2d((void *)P->tp.blksrc, P->blksrc.data(), P->blksrc.size() * 4);
  h2d((void *)P->tp.pairoff, P->pairoff.data(), P->pairoff.size() * 8);
  h2d((void *)P->tp.pairblk, P->pairblk.data(), P->pairblk.size() * 4);
  h2d((void *)P->tp.zmean, P->zmean.data(), P->zmean.size() * 8);
  if (!P->local_dev) h2d(P->rec, P->loc.rec.data(), P->loc.rec.size() * 8);
  h2d(P->roff, P->loc.off.data(), P->loc.off.size() * 8);
  if (P->local_dev) {
    const hho_mesh *m = P->mesh;
    const LocalGeom &g = P->lg;
    const LocalGeomHost &H = P->lgeo;
    h2d((void *)g.csign, m->csign.data(), m->csign.size() * 8);
    h2d((void *)g.fptr, m->fptr.data(), m->fptr.size() * 8);
    h2d((void *)g.fvtx, m->fvtx.data(), m->fvtx.size() * 8);
    h2d((void *)g.verts, m->verts.data(), m->verts.size() * 8);
    h2d((void *)g.rptr, H.rptr.data(), H.rptr.size() * 8);
    h2d((void *)g.ring, H.ring.data(), H.ring.size() * 8);
    h2d((void *)g.cbox, m->cbox.data(), m->cbox.size());
    h2d((void *)g.clo, m->clo.data(), m->clo.size() * 8);
    h2d((void *)g.chi, m->chi.data(), m->chi.size() * 8);
    h2d((void *)g.apex, H.apex.data(), H.apex.size() * 8);
    h2d((void *)g.ccen, m->ccen.data(), m->ccen.size() * 8);
    h2d((void *)g.cdiam, m->cdiam.data(), m->cdiam.size() * 8);
    h2d((void *)g.fcen, m->fcen.data(), m->fcen.size() * 8);
    h2d((void *)g.fdiam, m->fdiam.data(), m->fdiam.size() * 8);
    h2d((void *)g.fnrm, m->fnrm.data(), m->fnrm.size() * 8);
    h2d((void *)g.ft1, m->ft1.data(), m->ft1.size() * 8);
    h2d((void *)g.ft2, m->ft2.data(), m->ft2.size() * 8);
    h2d((void *)g.fbc, m->fbc.data(), m->fbc.size());
    h2d((void *)g.eta, P->cell_eta_dev.data(), P->cell_eta_dev.size() * 8);
    h2d((void *)g.glt, H.glt.data(), H.glt.size() * 8);
    h2d((void *)g.glw, H.glw.data(), H.glw.size() * 8);
    h2d((void *)g.EC, H.EC.data(), H.EC.size() * 4);
    h2d((void *)g.EF, H.EF.data(), H.EF.size() * 4);
    h2d((void *)g.mf, P->dmom.mf.data(), P->dmom.mf.size() * 8);
    h2d((void *)g.fd, P->dmom.fd.data(), P->dmom.fd.size() * 8);
    h2d((void *)g.foff, P->dmom.foff.data(), P->dmom.foff.size() * 8);
    if (!P->user_rhs.empty()) {
      h2d(P->d_user_rhs, P->user_rhs.data(), P->user_rhs.size() * 8);
      h2d(P->d_user_off, P->user_off.data(), P->user_off.size() * 8);
    }
  }
  HIPCHK(hipMemsetAsync(P->err, 0, 8 * sizeof(int), s));
  // nullspace vector (constant pressure on the level-0 mean modes)
  const LevelInfo &L0 = P->lev[0];
  P->zhost.assign(L0.N, 0.0);
  if (P->border)
    for (int64_t c = 0; c < P->mesh->nc; ++c) P->zhost[L0.nface + c * L0.t] = P->zmean[c];
  h2d(P->zvec, P->zhost.data(), P->zhost.size() * 8);
  if (P->nseg > 0) {
    h2d(P->dseg, P->hseg.data(), P->hseg.size() * sizeof(SegInfo));
    h2d(P->dchunks, P->hchunks.data(), P->hchunks.size() * sizeof(SegChunk));
    h2d(P->dchunk_ptr, P->hchunk_ptr.data(), P->hchunk_ptr.size() * 4);
    for (int l = 1; l < P->nlev; ++l) {
      const SegLevel &S = P->segl[l];
      h2d(S.seg, S.hseg.data(), S.hseg.size() * sizeof(SegInfo));
      h2d(S.ch, S.hch.data(), S.hch.size() * sizeof(SegChunk));
      h2d(S.ptr, S.hptr.data(), S.hptr.size() * 4);
    }
  }
  if (P->ilu_on)
    for (int l = 0; l < P->nlev; ++l) {
      if (!ilu_level(P, l)) continue;
      const IluHost &H = P->ilu[l];
      h2d((void *)H.dev.gptr, H.gptr.data(), H.gptr.size() * 8);
      h2d((void *)H.dev.gcol, H.gcol.data(), H.gcol.size() * 4);
      h2d((void *)H.dev.voff, H.voff.data(), H.voff.size() * 8);
      h2d((void *)H.dev.diag, H.diag.data(), H.diag.size() * 8);
      h2d(H.d_lrows, H.lrows.data(), H.lrows.size() * 4);
      h2d(H.d_urows, H.urows.data(), H.urows.size() * 4);
    }
  if (P->coarse_direct) {
    const NdHost &H = P->nd;
    const NdDev &D = P->ndd;
    h2d((void *)D.m, H.m.data(), H.m.size() * 4);
    h2d((void *)D.nfs, H.nfs.data(), H.nfs.size() * 4);
    h2d((void *)D.child, H.child.data(), H.child.size() * 4);
    h2d((void *)D.off, H.off.data(), H.off.size() * 8);
    h2d((void *)D.voff, H.voff.data(), H.voff.size() * 8);
    h2d((void *)D.dofoff, H.dofoff.data(), H.dofoff.size() * 8);
    h2d((void *)D.soff, H.soff.data(), H.soff.size() * 8);
    h2d((void *)D.dof, H.dof.data(), H.dof.size() * 4);
    h2d((void *)D.cmap, H.cmap.data(), H.cmap.size() * 4);
    h2d((void *)D.src, H.src.data(), H.src.size() * 8);
    h2d((void *)D.dst, H.dst.data(), H.dst.size() * 8);
    h2d((void *)D.hfront, H.hfront.data(), H.hfront.size() * 4);
    if (!H.tiles.empty()) h2d((void *)D.tiles, H.tiles.data(), H.tiles.size() * 4);
    h2d((void *)D.chunks, H.chunks.data(), H.chunks.size() * 4);
    h2d((void *)D.schunks, H.schunks.data(), H.schunks.size() * 4);
    h2d((void *)D.pins, H.pins.data(), H.pins.size() * 8);
    h2d((void *)D.segp, H.segp.data(), H.segp.size() * 8);
    h2d((void *)D.cseg, H.cseg.data(), H.cseg.size() * 4);
  }
  if (P->coarse_amg) {
    h2d(P->d_fdiag, P->fdiag.data(), P->fdiag.size() * 4);
    for (int l = 0; l < P->amgd.nlev; ++l) {
      const AmgHostLevel &H = P->amgh.levels[l];
      AmgDevLevel &G = P->amgd.lev[l];
      h2d((void *)G.rp, H.rp.data(), H.rp.size() * 4);
      h2d((void *)G.ci, H.ci.data(), H.ci.size() * 4);
      h2d((void *)G.diag, H.diag.data(), H.diag.size() * 4);
      if (H.nc > 0) {
        std::vector<int32_t> prow(H.pci.size());
        for (int i = 0; i < H.n; ++i)
          for (int e = H.prp[i]; e < H.prp[i + 1]; ++e) prow[e] = i;
        h2d((void *)G.prp, H.prp.data(), H.prp.size() * 4);
        h2d((void *)G.pci, H.pci.data(), H.pci.size() * 4);
        h2d((void *)G.prow, prow.data(), prow.size() * 4);
        h2d((void *)G.pgp, H.pgp.data(), H.pgp.size() * 4);
        h2d((void *)G.pgi, H.pgi.data(), H.pgi.size() * 4);
        h2d((void *)G.pself, H.pself.data(), H.pself.size() * 4);
        if (H.np1 > 0) {
          h2d((void *)G.p1row, H.p1row.data(), H.p1row.size() * 4);
          h2d((void *)G.qpp, H.qpp.data(), H.qpp.size() * 4);
          h2d((void *)G.qpa, H.qpa.data(), H.qpa.size() * 4);
          h2d((void *)G.qpb, H.qpb.data(), H.qpb.size() * 4);
          h2d((void *)G.p2src, H.p2src.data(), H.p2src.size() * 4);
        }
        h2d((void *)G.ptp, H.ptp.data(), H.ptp.size() * 4);
        h2d((void *)G.pti, H.pti.data(), H.pti.size() * 4);
        h2d((void *)G.pte, H.pte.data(), H.pte.size() * 4);
        h2d((void *)G.bpp, H.bpp.data(), H.bpp.size() * 4);
        h2d((void *)G.bpa, H.bpa.data(), H.bpa.size() * 4);
        h2d((void *)G.bpb, H.bpb.data(), H.bpb.size() * 4);
        h2d((void *)G.brp, H.brp.data(), H.brp.size() * 4);
        h2d((void *)G.bci, H.bci.data(), H.bci.size() * 4);
        h2d((void *)G.btp, H.btp.data(), H.btp.size() * 4);
        h2d((void *)G.bti, H.bti.data(), H.bti.size() * 4);
        h2d((void *)G.bte, H.bte.data(), H.bte.size() * 4);
        h2d((void *)G.cpp, H.cpp.data(), H.cpp.size() * 4);
        h2d((void *)G.cpa, H.cpa.data(), H.cpa.size() * 4);
        h2d((void *)G.cpb, H.cpb.data(), H.cpb.size() * 4);
      }
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  P->uploaded = true;
}

// the caller's right-hand-side moments (hho_set_moments) over the device build's
__global__ void k_user_rhs(int d, int nT, const int64_t *roff, const int64_t *uoff, const double *u, double *rec) {
  const int64_t c = blockIdx.x;
  const int64_t len = uoff[c + 1] - uoff[c];       // d nloc + nT
  const int64_t nloc = (len - nT) / d;
  double *dst = rec + roff[c] + nloc * nloc + (int64_t)d * nT * nloc;
  for (int64_t e = threadIdx.x; e < len; e += blockDim.x) dst[e] = u[uoff[c] + e];
}

// Whether the local operators are built on the device: options.local_build, and
// for AUTO the device build's limits (every rhs_u entry of a cell on its own
// thread of its workgroup, the cell's work arrays within the compute unit's LDS, quadrature
// within the node table).
static bool choose_local_device(hho_problem *P, int qdeg) {
  const int mode = P->opt.local_build;
  if (mode == HHO_LOCAL_HOST) return false;
  const int d = P->d, k = P->k;
  const int odeg = std::min(qdeg, 2 * k + 2);
  const int nT = dim_poly(d, k), nF = dim_poly(d - 1, k);
  const int nloc_max = nT + P->mesh->max_faces * nF;
  std::string why;
  if ((odeg + 4) / 2 >= kGlTable) why = "quadrature degree above the node table";
  if (why.empty() && d * nloc_max > kLocalThreads) why = "more velocity unknowns in a cell than threads";
  if (why.empty()) {
    build_local_geometry(P->mesh, k, qdeg, &P->lgeo);
    P->llds = local_lds(d, k, P->mesh->max_faces, P->lgeo.max_nq, P->lgeo.max_nqf);
    if (P->llds.bytes > kMaxLdsBytes - 2048) why = "a cell's work arrays exceed the LDS";
  }
  if (why.empty()) return true;
  if (mode == HHO_LOCAL_DEVICE) fail(HHO_E_INVALID_ARG, "local_build DEVICE: " + why);
  return false;
}

static void device_setup(hho_problem *P) {
  hipStream_t s = P->stream;
  const hho_mesh *m = P->mesh;
  const int64_t nc = m->nc;
  if (!P->uploaded) device_upload(P);
  HIPCHK(hipMemsetAsync(P->err, 0, 8 * sizeof(int), s));
  hipEvent_t ev[8], evl;
  for (auto &e : ev) HIPCHK(hipEventCreate(&e));
  HIPCHK(hipEventCreate(&evl));
  HIPCHK(hipEventRecord(evl, s));
  if (P->local_dev) {  // local operators of every cell, then the caller's moments if any
    launch_local(P->lg, P->llds, (int)nc, s);
    if (!P->user_rhs.empty())
      hipLaunchKernelGGL(k_user_rhs, dim3((unsigned)nc), dim3(256), 0, s, P->d, P->loc.nT, P->roff,
                         (const int64_t *)P->d_user_off, (const double *)P->d_user_rhs, P->rec);
  }
  HIPCHK(hipEventRecord(ev[0], s));
  LevelInfo &L0 = P->lev[0];
  // static condensation
  launch_condense(P->tp, P->cond, P->loc.nT, P->loc.nF, P->rec, P->roff, P->stage, L0.cpl, L0.spp, P->rhs_stage,
                  P->rhs + L0.nface, P->err, s, P->lds_condense, P->stage32);
  HIPCHK(hipEventRecord(ev[1], s));
  // assembly
  launch_assemble(P->tp, P->cond, L0.p, P->nnzb, P->stage, L0.bsr, P->rhs_stage, P->rhs, s);
  HIPCHK(hipEventRecord(ev[2], s));
  // coarse levels by extraction
  for (int l = 1; l < P->nlev; ++l) {
    const LevelInfo &A = P->lev[l - 1];
    LevelInfo &B = P->lev[l];
    launch_extract(P->tp, P->cond, P->nnzb, A.p, A.t, B.p, B.t, A.bsr, A.cpl, A.spp, B.bsr, B.cpl, B.spp, s);
  }
  HIPCHK(hipEventRecord(ev[3], s));
  // smoother patches (the condensation staging array is free now)
  const int Lc = P->nlev - 1;
  for (int l = 0; l < P->nlev; ++l) {
    LevelInfo &L = P->lev[l];
    if (!L.sinv || P->ilu_on) continue;
    size_t lds = patch_lds_bytes(P->d, P->cond, L.p, L.t, P->max_faces);
    launch_patch_setup(P->tp, P->cond, L.p, L.t, L.bsr, L.cpl, L.spp, L.sinv, L.xinv, L.sig, P->stage, P->err + 1,
                       s, lds, L.patch_threads);
  }
  for (int l = 0; l < P->nlev; ++l) {  // the paper's smoother: incomplete factors of the level operators
    if (!ilu_level(P, l)) continue;
    IluHost &H = P->ilu[l];
    launch_ilu_fill(P->tp, dlev64(P, l), H.dev, s);
    launch_ilu_factor(H.dev, H.d_lrows, H.lptr.data(), (int)H.lptr.size() - 1, H.maxrow, P->err + 5, s);
  }
  HIPCHK(hipEventRecord(ev[4], s));
  // coarse solver
  if (P->coarse_dense) {
    const int64_t n = P->dense_n;
    launch_fill<double>(n * 2 * n, 0.0, P->dense, s);
    launch_densify(P->tp, dlev64(P, Lc), P->border, P->dense, 2 * n, s);
    launch_eye_right(P->dense, n, 2 * n, s);
    for (int64_t kk = 0; kk < n; ++kk) launch_gj_step(P->dense, n, 2 * n, kk, P->colbuf, P->err + 2, s);
  }
  if (P->coarse_direct) {
    const LevelInfo &LC = P->lev[Lc];
    const int bs = LC.bs;
    launch_nd_factor(P->nd, P->ndd, dlev64(P, Lc), P->nnzb * bs * bs, P->ncf * P->d * LC.p * LC.t, P->err + 6, s);
  }
  if (P->coarse_amg) {
    const LevelInfo &LC = P->lev[Lc];
    bp_setup(P->tp, P->cond, P->d_fdiag, LC.bsr, LC.cpl, P->Sd, s);
    amg_numeric_setup(P->amgd, P->cond, P->d, LC.bs, P->nnzb, LC.bsr, P->amg_nu, P->err + 3, s);
  }
  // FP32 or bfloat16 copies for the mixed-precision V-cycle
  if (P->opt.precision != HHO_PREC_FP64) {
    for (int l = 0; l < Lc; ++l) {
      LevelInfo &L = P->lev[l];
      const int d = P->d;
      const int64_t nbsr = P->nnzb * L.bs * L.bs;
      const int64_t ncpl = P->ncf * d * L.p * (P->cond == HHO_COND_V ? L.t : 1);
      const int64_t nspp = P->cond == HHO_COND_V ? nc * L.t * L.t : 1;
      const int64_t nsinv = P->pairoff[nc] * L.bs * L.bs;
      const int64_t nxinv = P->cond == HHO_COND_V ? nc * L.t * L.t : P->ncf * d * L.p;
      const bool product = l == 0 && P->stage32;  // level-0 face blocks by the matrix-core product
      if (P->opt.precision == HHO_PREC_BF16) {
        if (product)
          launch_assemble32<bf16>(P->tp, P->cond, L.p, P->nnzb, P->stage32, L.bsr16, s);
        else
          launch_convert<bf16, double>(L.bsr, L.bsr16, nbsr, s);
        launch_convert<bf16, double>(L.cpl, L.cpl16, ncpl, s);
        if (P->cond == HHO_COND_V) launch_convert<bf16, double>(L.spp, L.spp16, nspp, s);
      } else {
        if (product)
          launch_assemble32<float>(P->tp, P->cond, L.p, P->nnzb, P->stage32, L.bsr32, s);
        else
          launch_convert<float, double>(L.bsr, L.bsr32, nbsr, s);
        launch_convert<float, double>(L.cpl, L.cpl32, ncpl, s);
        if (P->cond == HHO_COND_V) launch_convert<float, double>(L.spp, L.spp32, nspp, s);
      }
      launch_convert<float, double>(L.sinv, L.sinv32, nsinv, s);
      launch_convert<float, double>(L.xinv, L.xinv32, nxinv, s);
      if (P->cond != HHO_COND_V) launch_convert<float, double>(L.sig, L.sig32, nc, s);
    }
  }
  HIPCHK(hipEventRecord(ev[5], s));
  HIPCHK(hipStreamSynchronize(s));
  check_device_error(P, "setup");
  float ms;
  for (int i = 0; i < 5; ++i) {
    HIPCHK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    P->timings[i] = ms;
  }
  HIPCHK(hipEventElapsedTime(&ms, evl, ev[0]));
  P->timings[9] = ms;
  for (auto &e : ev) HIPCHK(hipEventDestroy(e));
  HIPCHK(hipEventDestroy(evl));
  int herr[8];
  HIPCHK(hipMemcpy(herr, P->err, sizeof(herr), hipMemcpyDeviceToHost));
  if (herr[4] > 0)
    fail(HHO_E_LOCAL_SINGULAR, "local build: degenerate basis or non-SPD reconstruction stiffness in cell " +
                                   std::to_string(herr[4] - 1));
  if (herr[4] < 0) fail(HHO_E_LOCAL_SINGULAR, "local build: degenerate basis of face " + std::to_string(-herr[4] - 1));
  if (herr[0]) fail(HHO_E_LOCAL_SINGULAR, "static condensation: local block not SPD in cell " + std::to_string(herr[0] - 1));
  if (herr[1]) fail(HHO_E_LOCAL_SINGULAR, "smoother patch not invertible in cell " + std::to_string(herr[1] - 1));
  if (herr[2]) fail(HHO_E_LOCAL_SINGULAR, "coarsest-level matrix is singular");
  if (herr[3]) fail(HHO_E_LOCAL_SINGULAR, "AMG coarsest matrix is not SPD");
  if (herr[5]) fail(HHO_E_LOCAL_SINGULAR, "ILU smoother: zero pivot in row " + std::to_string(herr[5] - 1));
  if (herr[6])
    fail(HHO_E_LOCAL_SINGULAR, "sparse direct coarse solver: zero pivot in front " + std::to_string(herr[6] - 1));
}

// ------------------------------------------------------------ V-cycle
// z = (L U)^{-1} r with level l's incomplete factors
static void ilu_apply(hho_problem *P, int l, const double *r, double *z) {
  const IluHost &H = P->ilu[l];
  launch_ilu_apply(H.dev, H.d_lrows, H.lptr.data(), (int)H.lptr.size() - 1, H.d_urows, H.uptr.data(),
                   (int)H.uptr.size() - 1, r, z, P->stream);
}

// z_j = M v_j and w = S z_j on the coarsest level (M its smoother's preconditioner)
static void coarse_precond(hho_problem *P, const DLevel<double> &D, const DLevel<double> &Dq, const double *vj,
                           double *zj) {
  if (P->ilu_on) {
    ilu_apply(P, P->nlev - 1, vj, zj);
    launch_spmv<double>(P->tp, Dq, zj, nullptr, nullptr, P->cw, P->stream);
    return;
  }
  launch_precond<double>(P->tp, D, vj, nullptr, nullptr, P->czs0, P->czs1, P->max_faces, P->stream);
  launch_spmv<double>(P->tp, Dq, P->czs0, P->czs1, zj, P->cw, P->stream);
}

template <typename Prec>
static void smooth(hho_problem *P, int l) {
  using T = typename Prec::T;
  hipStream_t s = P->stream;
  const auto D = Prec::op(P, l);
  VBufs<T> &V = Prec::vb(P, l);
  const int m = P->opt.smooth_its;
  const int64_t n = D.N;
  const bool learned = l == 0 && P->learned_on;
  if (learned) {  // learned direction from the residual at the start of the step
    const MlpDims &md = P->md;
    launch_mlp_windows<T>(P->tp, md, V.r, P->mlp_X, P->mlp_sc, s);
    launch_mlp_forward(P->tp.nf, md, P->mlp_X, nullptr, P->mlp_prm, P->mlp_w1b, P->mlp_w2b, nullptr, P->mlp_Y, s);
    launch_mlp_scatter<T>(P->tp, md, n, P->mlp_Y, P->mlp_sc, V.z3, s);
    launch_spmv<T>(P->tp, D, V.z3, nullptr, nullptr, V.w3, s);
  }
  KernelProbe *pr = &P->probe;
  bool ilu = false;
  if constexpr (std::is_same<T, double>::value) {
    if (P->ilu_on) {  // the paper's smoother: GMRES(2) right-preconditioned by the level's ILU
      ilu = true;
      ilu_apply(P, l, V.r, V.z1);
      HHO_PROBED(pr, HHO_PROBE_OPERATOR, l, s, launch_spmv<T>(P->tp, D, V.z1, nullptr, nullptr, V.w1, s));
      if (m == 2) {
        ilu_apply(P, l, V.w1, V.z2);
        HHO_PROBED(pr, HHO_PROBE_OPERATOR, l, s, launch_spmv<T>(P->tp, D, V.z2, nullptr, nullptr, V.w2, s));
      }
    }
  }
  if (!ilu) {
    HHO_PROBED(pr, HHO_PROBE_SMOOTHER, l, s, launch_precond<T>(P->tp, D, V.r, nullptr, nullptr, V.zs0, V.zs1, P->max_faces, s));
    HHO_PROBED(pr, HHO_PROBE_OPERATOR, l, s, launch_spmv<T>(P->tp, D, V.zs0, V.zs1, V.z1, V.w1, s));
    if (m == 2) {
      HHO_PROBED(pr, HHO_PROBE_SMOOTHER, l, s, launch_precond<T>(P->tp, D, V.w1, nullptr, nullptr, V.zs0, V.zs1, P->max_faces, s));
      HHO_PROBED(pr, HHO_PROBE_OPERATOR, l, s, launch_spmv<T>(P->tp, D, V.zs0, V.zs1, V.z2, V.w2, s));
    }
  }
  if (P->nseg > 0) {  // batch: every member takes its own minimal-residual step
    const SegLevel &S = P->segl[l];
    launch_seg_mr<T>(S.G(), S.ch, S.seg, P->nseg, S.ptr, m, V.z1, V.z2, learned ? V.z3 : nullptr, V.w1, V.w2,
                     learned ? V.w3 : nullptr, V.w, V.r, P->seg_partial, P->seg_y, s);
    return;
  }
  if (learned) {
    launch_mr3<T>(n, m, V.z1, V.z2, V.z3, V.w1, V.w2, V.w3, V.w, V.r, P->partial, P->lev[l].y, s);
    return;
  }
  launch_mr2_dots<T>(n, m, V.w1, V.w2, V.r, P->partial, P->lev[l].y, s);
  launch_mr2_update<T>(n, m, P->lev[l].y, V.z1, V.z2, V.w1, V.w2, V.w, V.r, s);
}

static void coarse_solve(hho_problem *P);

// MG_V(l, b, 0): input lev[l] b, output lev[l] w
template <typename Prec>
static void vcycle(hho_problem *P, int l) {
  using T = typename Prec::T;
  hipStream_t s = P->stream;
  const int Lc = P->nlev - 1;
  const auto D = Prec::op(P, l);
  VBufs<T> &V = Prec::vb(P, l);
  const LevelInfo &A = P->lev[l], &B = P->lev[l + 1];
  const int d = P->d, nf = (int)P->mesh->nf, nc = (int)P->mesh->nc;
  launch_fill<T>(D.N, (T)0, V.w, s);
  launch_copy<T>(D.N, V.b, V.r, s);
  smooth<Prec>(P, l);
  if (l + 1 == Lc) {
    launch_restrict<double, T>(d, nf, nc, A.p, A.t, B.p, B.t, V.r, P->lev[Lc].v64.b, s);
    coarse_solve(P);
    launch_prolong_add<double, T>(d, nf, nc, A.p, A.t, B.p, B.t, P->lev[Lc].v64.w, V.w, s);
  } else {
    VBufs<T> &W = Prec::vb(P, l + 1);
    launch_restrict<T, T>(d, nf, nc, A.p, A.t, B.p, B.t, V.r, W.b, s);
    vcycle<Prec>(P, l + 1);
    launch_prolong_add<T, T>(d, nf, nc, A.p, A.t, B.p, B.t, W.w, V.w, s);
  }
  launch_residual<T>(P->tp, D, V.b, V.w, V.r, s);
  smooth<Prec>(P, l);
}

static void read_state(hho_problem *P, GmresState *dst) {
  HIPCHK(hipMemcpyAsync(P->h_st, dst, sizeof(GmresState), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
}

static void set_rtol(hho_problem *P, GmresState *st, double rtol) {
  HIPCHK(hipMemcpyAsync(&st->rtol, &rtol, sizeof(double), hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
}

// GMRES state of every segment reset, with its tolerance
__global__ void k_seg_init(int np, GmresState *st, double rtol) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  st[p].rtol = rtol;
  st[p].done = 0;
  st[p].nan = 0;
  st[p].its = 0;
  st[p].j = 0;
}

static bool read_flag(hho_problem *P, const int *flag) {
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return h != 0;
}

// The coarse GMRES of a batch: one Krylov process per member over its slice of
// the coarsest level (the same steps as coarse_solve: classical Gram-Schmidt once
// with the new norm taken after the subtraction, restarts from the true
// residual), so no member's coarse correction depends on another member's
// residual.  The preconditioner acts on the whole union, which is block
// diagonal; once every member has converged the queued operator kernels return
// at once.
static void coarse_solve_seg(hho_problem *P) {
  hipStream_t s = P->stream;
  const int Lc = P->nlev - 1, np = P->nseg;
  LevelInfo &L = P->lev[Lc];
  VBufs<double> &V = L.v64;
  const SegLevel &S = P->segl[Lc];
  const int G = S.G();
  const DLevel<double> D = dlev64(P, Lc);
  const int64_t n = L.N;
  const int R = P->opt.coarse_restart;
  GmresState *st = P->csst;
  DLevel<double> Dq = D;
  Dq.skip = P->call_done;
  launch_fill<double>(n, 0.0, V.w, s);
  hipLaunchKernelGGL(k_seg_init, dim3((np + 63) / 64), dim3(64), 0, s, np, st, P->opt.coarse_rtol);
  launch_seg_sumsq(G, S.ch, S.seg, V.b, P->seg_partial, s);
  launch_seg_norm_finish(np, S.ptr, G, P->seg_partial, st, P->csdone, 1, s);
  launch_seg_scale(G, S.ch, S.seg, V.b, st, P->cV, s);
  launch_seg_all_done(np, P->csdone, P->call_done, s);
  bool all = read_flag(P, P->call_done);
  int its = 0;
  const int chunk = 6;
  while (!all && its < P->opt.coarse_max_it) {
    const int jmax = std::min(R, P->opt.coarse_max_it - its);
    int jn = 0;
    for (int j = 0; j < jmax; ++j) {
      double *vj = P->cV + (int64_t)j * n, *zj = P->cZ + (int64_t)j * n;
      if (P->coarse_amg) {
        bp_apply(P->tp, P->amgd, L.nface, L.cpl, P->Sd, vj, zj, P->amg_nu, s, P->call_done);
        HHO_PROBED(&P->probe, HHO_PROBE_COARSE_OPERATOR, Lc, s,
                   launch_spmv<double>(P->tp, Dq, zj, nullptr, nullptr, P->cw, s));
      } else {
        coarse_precond(P, D, Dq, vj, zj);
      }
      launch_seg_arnoldi(0, G, S.ch, S.seg, np, S.ptr, j, P->cV, n, P->cw, P->seg_partial, st, P->csdone, 0, s);
      launch_seg_arnoldi(2, G, S.ch, S.seg, np, S.ptr, j, P->cV, n, P->cw, P->seg_partial, st, P->csdone, 0, s);
      launch_seg_scale(G, S.ch, S.seg, P->cw, st, P->cV + (int64_t)(j + 1) * n, s);
      launch_seg_all_done(np, P->csdone, P->call_done, s);
      jn = j + 1;
      if ((j + 1) % chunk == 0 || j + 1 == jmax) {
        all = read_flag(P, P->call_done);
        if (all) break;
      }
    }
    its += jn;
    launch_seg_solve_ls(np, st, s);
    launch_seg_combine(G, S.ch, S.seg, P->cZ, n, st, V.w, s);
    if (all || its >= P->opt.coarse_max_it) break;
    // restart the unconverged members from their true residuals; a converged one
    // stays done, as a single problem's coarse solve stops at its estimate
    launch_residual<double>(P->tp, D, V.b, V.w, P->cr, s);
    launch_seg_sumsq(G, S.ch, S.seg, P->cr, P->seg_partial, s);
    launch_seg_norm_finish(np, S.ptr, G, P->seg_partial, st, P->csdone, 2, s);
    launch_seg_scale(G, S.ch, S.seg, P->cr, st, P->cV, s);
    launch_seg_all_done(np, P->csdone, P->call_done, s);
    all = read_flag(P, P->call_done);
  }
  P->coarse_its += its;
}

// The coarse GMRES inside a captured V-cycle: one cycle of at most
// coarse_restart columns with no host read and no restart; once the process (or,
// in a batch, every member's) has converged the remaining columns' kernels return
// at once on the device, and the correction is formed from the columns taken.
// While the eager solve does not restart, the two take the same steps.
static void coarse_solve_fixed(hho_problem *P) {
  hipStream_t s = P->stream;
  const int Lc = P->nlev - 1;
  LevelInfo &L = P->lev[Lc];
  VBufs<double> &V = L.v64;
  const DLevel<double> D = dlev64(P, Lc);
  const int64_t n = L.N;
  const int R = std::min(P->opt.coarse_restart, P->opt.coarse_max_it);
  launch_fill<double>(n, 0.0, V.w, s);
  if (P->nseg > 0) {
    const int np = P->nseg;
    const SegLevel &S = P->segl[Lc];
    const int G = S.G();
    GmresState *st = P->csst;
    DLevel<double> Dq = D;
    Dq.skip = P->call_done;
    hipLaunchKernelGGL(k_seg_init, dim3((np + 63) / 64), dim3(64), 0, s, np, st, P->opt.coarse_rtol);
    launch_seg_sumsq(G, S.ch, S.seg, V.b, P->seg_partial, s);
    launch_seg_norm_finish(np, S.ptr, G, P->seg_partial, st, P->csdone, 1, s);
    launch_seg_scale(G, S.ch, S.seg, V.b, st, P->cV, s);
    launch_seg_all_done(np, P->csdone, P->call_done, s);
    for (int j = 0; j < R; ++j) {
      double *vj = P->cV + (int64_t)j * n, *zj = P->cZ + (int64_t)j * n;
      if (P->coarse_amg) {
        bp_apply(P->tp, P->amgd, L.nface, L.cpl, P->Sd, vj, zj, P->amg_nu, s, P->call_done);
        launch_spmv<double>(P->tp, Dq, zj, nullptr, nullptr, P->cw, s);
      } else {
        coarse_precond(P, D, Dq, vj, zj);
      }
      launch_seg_arnoldi(0, G, S.ch, S.seg, np, S.ptr, j, P->cV, n, P->cw, P->seg_partial, st, P->csdone, 0, s);
      launch_seg_arnoldi(2, G, S.ch, S.seg, np, S.ptr, j, P->cV, n, P->cw, P->seg_partial, st, P->csdone, 0, s);
      launch_seg_scale(G, S.ch, S.seg, P->cw, st, P->cV + (int64_t)(j + 1) * n, s);
      launch_seg_all_done(np, P->csdone, P->call_done, s);
    }
    launch_seg_solve_ls(np, st, s);
    launch_seg_combine(G, S.ch, S.seg, P->cZ, n, st, V.w, s);
    return;
  }
  GmresState *st = P->cst;
  DLevel<double> Dq = D;
  Dq.skip = &st->done;
  launch_norm_init<double>(n, V.b, P->partial, st, 1, s);
  launch_scale<double>(n, V.b, &st->inv_hnext, P->cV, s);
  for (int j = 0; j < R; ++j) {
    double *vj = P->cV + (int64_t)j * n;
    if (P->coarse_amg) {
      bp_apply(P->tp, P->amgd, L.nface, L.cpl, P->Sd, vj, P->cZ + (int64_t)j * n, P->amg_nu, s, &st->done);
      launch_spmv<double>(P->tp, Dq, P->cZ + (int64_t)j * n, nullptr, nullptr, P->cw, s);
    } else {
      coarse_precond(P, D, Dq, vj, P->cZ + (int64_t)j * n);
    }
    if (j + 2 <= 64) {
      launch_arnoldi_cgs1<double>(n, j, P->cV, n, P->cw, P->partial, st, s);
    } else {
      launch_arnoldi_dots<double>(n, j, P->cV, n, P->cw, P->partial, st, s);
      launch_arnoldi_update<double>(n, j, P->cV, n, P->cw, P->partial, st, 2, 0, s);
      launch_scale<double>(n, P->cw, &st->inv_hnext, P->cV + (int64_t)(j + 1) * n, s);
    }
  }
  launch_gmres_solve_ls(st, s);
  launch_gmres_combine<double>(n, P->cZ, n, st, V.w, s);
}

// coarsest level: lev[Lc].v64.b -> lev[Lc].v64.w (FP64)
static void coarse_solve(hho_problem *P) {
  hipStream_t s = P->stream;
  const int Lc = P->nlev - 1;
  LevelInfo &L = P->lev[Lc];
  VBufs<double> &V = L.v64;
  if (P->coarse_dense) {
    launch_dense_matvec(P->dense, P->dense_n, 2 * P->dense_n, P->border, V.b, V.w, s);
    return;
  }
  if (P->coarse_direct) {
    launch_nd_solve(P->nd, P->ndd, L.nface, L.t, P->tp.zmean, V.b, V.w, s, &P->probe);
    return;
  }
  if (P->in_capture) {
    coarse_solve_fixed(P);
    return;
  }
  if (P->nseg > 0) {
    coarse_solve_seg(P);
    return;
  }
  const DLevel<double> D = dlev64(P, Lc);
  const int64_t n = L.N;
  const int R = P->opt.coarse_restart;
  GmresState *st = P->cst;
  DLevel<double> Dq = D;
  Dq.skip = &st->done;
  launch_fill<double>(n, 0.0, V.w, s);
  launch_norm_init<double>(n, V.b, P->partial, st, 1, s);
  launch_scale<double>(n, V.b, &st->inv_hnext, P->cV, s);
  read_state(P, st);
  int its = 0;
  const int chunk = 6;
  while (!P->h_st->done && its < P->opt.coarse_max_it) {
    // one restart cycle; the host looks at the device state every `chunk` columns
    const int jmax = std::min(R, P->opt.coarse_max_it - its);
    for (int j = 0; j < jmax; ++j) {
      double *vj = P->cV + (int64_t)j * n;
      // once the process has converged inside the chunk, the remaining queued
      // iterations' preconditioner and operator kernels return at once (the
      // Arnoldi kernels test the same flag)
      if (P->coarse_amg) {
        bp_apply(P->tp, P->amgd, L.nface, L.cpl, P->Sd, vj, P->cZ + (int64_t)j * n, P->amg_nu, s, &st->done);
        HHO_PROBED(&P->probe, HHO_PROBE_COARSE_OPERATOR, Lc, s,
                   launch_spmv<double>(P->tp, Dq, P->cZ + (int64_t)j * n, nullptr, nullptr, P->cw, s));
      } else {
        coarse_precond(P, D, Dq, vj, P->cZ + (int64_t)j * n);
      }
      // coarse GMRES: classical Gram-Schmidt once (its target is a 1e-3 reduction),
      // the new norm from |w|^2 - |h|^2, the next basis vector written directly
      // (while the j + 2 sums fit the 64 slots of the update pass)
      if (j + 2 <= 64) {
        launch_arnoldi_cgs1<double>(n, j, P->cV, n, P->cw, P->partial, st, s);
      } else {
        launch_arnoldi_dots<double>(n, j, P->cV, n, P->cw, P->partial, st, s);
        launch_arnoldi_update<double>(n, j, P->cV, n, P->cw, P->partial, st, 2, 0, s);
        launch_scale<double>(n, P->cw, &st->inv_hnext, P->cV + (int64_t)(j + 1) * n, s);
      }
      if ((j + 1) % chunk == 0 || j + 1 == jmax) {
        read_state(P, st);
        if (P->h_st->done) break;
      }
    }
    its += P->h_st->j;
    launch_gmres_solve_ls(st, s);
    launch_gmres_combine<double>(n, P->cZ, n, st, V.w, s);
    if (P->h_st->nan) fail(HHO_E_BREAKDOWN, "coarse GMRES: non-finite value");
    if (P->h_st->res <= P->h_st->rtol * P->h_st->bnorm || its >= P->opt.coarse_max_it) break;
    // restart from the true residual
    launch_residual<double>(P->tp, D, V.b, V.w, P->cr, s);
    launch_norm_init<double>(n, P->cr, P->partial, st, 0, s);
    launch_scale<double>(n, P->cr, &st->inv_hnext, P->cV, s);
    read_state(P, st);
  }
  P->coarse_its += its;
}

// The V-cycle from lev[0]'s input vector (v64.b, or v32.b below FP64) to its
// output (.w); the part of apply_vcycle that a HIP graph captures.
static void vcycle_body(hho_problem *P) {
  if (P->nlev == 1)
    coarse_solve(P);
  else if (P->opt.precision == HHO_PREC_BF16)
    vcycle<PrecB16>(P, 0);
  else if (P->opt.precision == HHO_PREC_FP32)
    vcycle<PrecF32>(P, 0);
  else
    vcycle<PrecF64>(P, 0);
}

void drop_graph(hho_problem *P) {
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
  P->gkey = -1;
}

// what the captured kernels depend on besides the workspace addresses
static int64_t graph_key(const hho_problem *P) {
  return (((((int64_t)P->opt.precision * 2 + (P->learned_on ? 1 : 0)) * 4 + P->opt.smooth_its) * 128 +
           P->opt.coarse_restart) * 4096 + P->opt.coarse_max_it) * 4 + P->amg_nu;
}

// Replays the captured V-cycle on the library's stream, capturing it first
// (again after an option that changes its kernels).  The capture records every
// launch of the V-cycle from a stream of the library's own (the caller's may be
// the legacy stream, which cannot be captured); probes are off while capturing.
static void vcycle_graph(hho_problem *P) {
  hipStream_t s = P->stream;
  if (!P->gexec || P->gkey != graph_key(P)) {
    drop_graph(P);
    if (!P->cap_stream) HIPCHK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    const unsigned mask = P->probe.mask;
    P->probe.mask = 0;
    P->in_capture = true;
    P->stream = P->cap_stream;
    hipError_t e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      vcycle_body(P);
      e = hipStreamEndCapture(P->cap_stream, &P->graph);
    }
    P->stream = s;
    P->in_capture = false;
    P->probe.mask = mask;
    HIPCHK(e);
    HIPCHK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
    P->gkey = graph_key(P);
  }
  HIPCHK(hipGraphLaunch(P->gexec, s));
}

// x = V-cycle(b) on level 0, b and x FP64 (device)
static void apply_vcycle(hho_problem *P, const double *b, double *x) {
  hipStream_t s = P->stream;
  LevelInfo &L0 = P->lev[0];
  const bool low = P->nlev > 1 && P->opt.precision != HHO_PREC_FP64;
  if (low)
    launch_convert<float, double>(b, L0.v32.b, L0.N, s);
  else
    launch_copy<double>(L0.N, b, L0.v64.b, s);
  if (P->graph_on)
    vcycle_graph(P);
  else
    vcycle_body(P);
  if (low)
    launch_convert<double, float>(L0.v32.w, x, L0.N, s);
  else
    launch_copy<double>(L0.N, L0.v64.w, x, s);
}

// ------------------------------------------------------------ FGMRES
// Flexible GMRES with one Krylov process per segment (problem) of a batch: the
// V-cycle and the operator act on the whole disjoint union (block diagonal),
// the Arnoldi reductions, Hessenberg columns, Givens rotations, restarts and
// convergence tests are per segment.  Converged segments stop contributing.

// relative residual estimate and Arnoldi step count of every segment
__global__ void k_seg_hist(int np, const GmresState *st, double *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double bn = st[p].bnorm;
  out[2 * p] = bn > 0 ? st[p].res / bn : 0.0;
  out[2 * p + 1] = (double)st[p].its;
}

// appends the estimate of every segment that took an Arnoldi step since the last call
static void record_seg_hist(hho_problem *P, std::vector<int> &last_its) {
  const int np = P->nseg;
  hipLaunchKernelGGL(k_seg_hist, dim3((np + 63) / 64), dim3(64), 0, P->stream, np, (const GmresState *)P->sst,
                     P->seg_hist);
  std::vector<double> h(2 * np);
  HIPCHK(hipMemcpyAsync(h.data(), P->seg_hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  for (int q = 0; q < np; ++q) {
    const int its = (int)h[2 * q + 1];
    if (its > last_its[q]) P->seg_hist_h[q].push_back(h[2 * q]);
    last_its[q] = its;
  }
}

static int read_seg_done(hho_problem *P) {
  std::vector<int> d(P->nseg);
  HIPCHK(hipMemcpyAsync(d.data(), P->sdone, P->nseg * sizeof(int), hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  int nd = 0;
  for (int x : d) nd += x != 0;
  return nd;
}

static int fgmres_batched(hho_problem *P, double *x_out, int *iters, double *hist, int hist_cap,
                          double *final_rel) {
  hipStream_t s = P->stream;
  const DLevel<double> D = dlev64(P, 0);
  const int64_t n = D.N;
  const int R = P->opt.restart, np = P->nseg, G = (int)P->hchunks.size();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  P->coarse_its = 0;
  launch_copy<double>(n, P->rhs, P->ob, s);
  if (P->border)
    launch_seg_project(np, P->dchunk_ptr, G, P->dchunks, P->dseg, P->zvec, P->ob, P->seg_partial, P->seg_ratio, s);
  hipLaunchKernelGGL(k_seg_init, dim3((np + 63) / 64), dim3(64), 0, s, np, P->sst, P->opt.rtol);
  launch_fill<double>(n, 0.0, P->ox, s);
  launch_seg_sumsq(G, P->dchunks, P->dseg, P->ob, P->seg_partial, s);
  launch_seg_norm_finish(np, P->dchunk_ptr, G, P->seg_partial, P->sst, P->sdone, 1, s);
  launch_seg_scale(G, P->dchunks, P->dseg, P->ob, P->sst, P->oV, s);
  int ndone = read_seg_done(P);
  int its = 0, nvc = 0;
  double vc_ms = 0;
  std::vector<hipEvent_t> ev;  // V-cycle start/end pairs, read after the solve
  if (hist && hist_cap > 0) hist[0] = 1.0;
  P->seg_hist_h.assign(np, std::vector<double>(1, 1.0));
  std::vector<int> last_its(np, 0);
  while (ndone < np && its < P->opt.max_it) {
    for (int j = 0; j < R && its < P->opt.max_it; ++j) {
      double *vj = P->oV + (int64_t)j * n, *zj = P->oZ + (int64_t)j * n;
      hipEvent_t va, vb;
      HIPCHK(hipEventCreate(&va));
      HIPCHK(hipEventCreate(&vb));
      ev.push_back(va);
      ev.push_back(vb);
      HIPCHK(hipEventRecord(va, s));
      apply_vcycle(P, vj, zj);
      HIPCHK(hipEventRecord(vb, s));
      ++nvc;
      launch_spmv<double>(P->tp, D, zj, nullptr, nullptr, P->ow, s);
      for (int mode = 0; mode < 3; ++mode)
        launch_seg_arnoldi(mode, G, P->dchunks, P->dseg, np, P->dchunk_ptr, j, P->oV, n, P->ow, P->seg_partial,
                           P->sst, P->sdone, 1, s);
      launch_seg_scale(G, P->dchunks, P->dseg, P->ow, P->sst, P->oV + (int64_t)(j + 1) * n, s);
      ++its;
      if (P->opt_seg_hist) record_seg_hist(P, last_its);
      ndone = read_seg_done(P);  // one small read per (batch-wide, heavy) iteration
      if (ndone == np) break;
    }
    launch_seg_solve_ls(np, P->sst, s);
    launch_seg_combine(G, P->dchunks, P->dseg, P->oZ, n, P->sst, P->ox, s);
    // true residual per segment; restart the unconverged ones from it
    launch_residual<double>(P->tp, D, P->ob, P->ox, P->or_, s);
    launch_seg_sumsq(G, P->dchunks, P->dseg, P->or_, P->seg_partial, s);
    launch_seg_norm_finish(np, P->dchunk_ptr, G, P->seg_partial, P->sst, P->sdone, 0, s);
    launch_seg_scale(G, P->dchunks, P->dseg, P->or_, P->sst, P->oV, s);
    ndone = read_seg_done(P);
  }
  if (P->border)
    launch_seg_project(np, P->dchunk_ptr, G, P->dchunks, P->dseg, P->zvec, P->ox, P->seg_partial, P->seg_ratio, s);
  if (x_out) launch_copy<double>(n, P->ox, x_out, s);
  HIPCHK(hipEventRecord(e1, s));
  // per-segment results
  std::vector<GmresState> hs(np);
  HIPCHK(hipMemcpyAsync(hs.data(), P->sst, np * sizeof(GmresState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  P->seg_its.assign(np, 0);
  P->seg_rel.assign(np, 0.0);
  double worst = 0;
  bool nan = false;
  for (int q = 0; q < np; ++q) {
    P->seg_its[q] = hs[q].its;
    P->seg_rel[q] = hs[q].bnorm > 0 ? hs[q].beta / hs[q].bnorm : 0.0;
    worst = std::max(worst, P->seg_rel[q]);
    nan = nan || hs[q].nan;
  }
  if (nan) fail(HHO_E_BREAKDOWN, "batched FGMRES: non-finite value");
  float ms;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  for (size_t q = 0; q + 1 < ev.size(); q += 2) {
    float vms;
    HIPCHK(hipEventElapsedTime(&vms, ev[q], ev[q + 1]));
    vc_ms += vms;
  }
  for (hipEvent_t e : ev) HIPCHK(hipEventDestroy(e));
  P->timings[5] = ms;
  P->timings[6] = vc_ms;
  P->timings[7] = nvc;
  P->timings[8] = (double)P->coarse_its;
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  check_device_error(P, "solve");
  int its_max = 0;
  for (int q = 0; q < np; ++q) its_max = std::max(its_max, P->seg_its[q]);
  if (iters) *iters = its_max;
  if (final_rel) *final_rel = worst;
  if (hist && hist_cap > 1) hist[std::min(its_max, hist_cap - 1)] = worst;
  return ndone == np ? HHO_OK : HHO_E_NOT_CONVERGED;
}

static int fgmres(hho_problem *P, double *x_out, int *iters, double *hist, int hist_cap, double *final_rel) {
  hipStream_t s = P->stream;
  const DLevel<double> D = dlev64(P, 0);
  const int64_t n = D.N;
  const int R = P->opt.restart;
  GmresState *st = P->ost;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  P->coarse_its = 0;
  // b <- b - (b.z / z.z) z  (consistent right-hand side when the pressure is defined up to a constant)
  launch_copy<double>(n, P->rhs, P->ob, s);
  if (P->border) {
    launch_dot<double>(n, P->ob, P->zvec, P->partial, P->scal + 0, s);
    launch_dot<double>(n, P->zvec, P->zvec, P->partial, P->scal + 1, s);
    launch_axpy_ratio<double>(n, P->scal, -1.0, P->zvec, P->ob, s);
  }
  set_rtol(P, st, P->opt.rtol);
  launch_fill<double>(n, 0.0, P->ox, s);
  launch_norm_init<double>(n, P->ob, P->partial, st, 1, s);
  launch_scale<double>(n, P->ob, &st->inv_hnext, P->oV, s);
  read_state(P, st);
  const double bnorm = P->h_st->bnorm;
  int its = 0, nh = 0;
  if (hist && hist_cap > 0) hist[nh++] = 1.0;
  bool converged = bnorm == 0.0;
  double rel = 0.0;
  int nvc = 0;
  double vc_ms = 0;
  hipEvent_t va, vb;
  HIPCHK(hipEventCreate(&va));
  HIPCHK(hipEventCreate(&vb));
  while (!converged && its < P->opt.max_it) {
    int j = 0;
    for (; j < R && its < P->opt.max_it; ++j) {
      double *vj = P->oV + (int64_t)j * n, *zj = P->oZ + (int64_t)j * n;
      HIPCHK(hipEventRecord(va, s));
      apply_vcycle(P, vj, zj);
      HIPCHK(hipEventRecord(vb, s));
      ++nvc;
      HHO_PROBED(&P->probe, HHO_PROBE_OUTER_OPERATOR, 0, s, launch_spmv<double>(P->tp, D, zj, nullptr, nullptr, P->ow, s));
      launch_arnoldi_dots<double>(n, j, P->oV, n, P->ow, P->partial, st, s);
      launch_arnoldi_update<double>(n, j, P->oV, n, P->ow, P->partial, st, 1, 1, s);
      launch_arnoldi_update<double>(n, j, P->oV, n, P->ow, P->partial, st, 2, 1, s);
      launch_scale<double>(n, P->ow, &st->inv_hnext, P->oV + (int64_t)(j + 1) * n, s);
      read_state(P, st);
      {
        float vms;
        HIPCHK(hipEventElapsedTime(&vms, va, vb));
        vc_ms += vms;
      }
      ++its;
      if (P->h_st->nan) fail(HHO_E_BREAKDOWN, "FGMRES: non-finite value");
      if (hist && nh < hist_cap) hist[nh++] = P->h_st->res / bnorm;
      if (P->h_st->done) {
        ++j;
        break;
      }
    }
    launch_gmres_solve_ls(st, s);
    launch_gmres_combine<double>(n, P->oZ, n, st, P->ox, s);
    // true residual
    launch_residual<double>(P->tp, D, P->ob, P->ox, P->or_, s);
    launch_norm_init<double>(n, P->or_, P->partial, st, 0, s);
    launch_scale<double>(n, P->or_, &st->inv_hnext, P->oV, s);
    read_state(P, st);
    rel = P->h_st->beta / bnorm;
    if (!std::isfinite(rel)) fail(HHO_E_BREAKDOWN, "FGMRES: non-finite residual");
    if (rel <= P->opt.rtol) converged = true;
  }
  // zero-mean pressure
  if (P->border) {
    launch_dot<double>(n, P->ox, P->zvec, P->partial, P->scal + 0, s);
    launch_dot<double>(n, P->zvec, P->zvec, P->partial, P->scal + 1, s);
    launch_axpy_ratio<double>(n, P->scal, -1.0, P->zvec, P->ox, s);
  }
  if (x_out) launch_copy<double>(n, P->ox, x_out, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  P->timings[5] = ms;
  P->timings[6] = vc_ms;
  P->timings[7] = nvc;
  HIPCHK(hipEventDestroy(va));
  HIPCHK(hipEventDestroy(vb));
  P->timings[8] = (double)P->coarse_its;
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  check_device_error(P, "solve");
  if (iters) *iters = its;
  if (final_rel) *final_rel = rel;
  return converged ? HHO_OK : HHO_E_NOT_CONVERGED;
}

}  // namespace hho

// ================================================================ C ABI
#define ABI_BEGIN try {
#define ABI_END                                                  \
  }                                                              \
  catch (const hho::Error &e) {                                  \
    hho::set_error(e.msg);                                       \
    return e.code;                                               \
  }                                                              \
  catch (const std::bad_alloc &) {                               \
    hho::set_error("host allocation failed");                    \
    return HHO_E_OOM;                                            \
  }                                                              \
  catch (const std::exception &e) {                              \
    hho::set_error(e.what());                                    \
    return HHO_E_INVALID_ARG;                                    \
  }

extern "C" {

const char *hho_last_error(void) { return hho::g_last_error.c_str(); }

void hho_options_default(hho_options *o) {
  if (!o) return;
  o->eta = 0;
  o->rtol = 1e-8;
  o->max_it = 1000;
  o->restart = 30;
  o->smooth_its = 2;
  o->precision = HHO_PREC_FP64;
  o->coarse_mode = HHO_COARSE_AUTO;
  o->coarse_rtol = 0.0;  // resolved per dimension at problem creation
  o->coarse_restart = 30;
  o->coarse_max_it = 300;
  o->quad_extra = 6;
  o->coarse_amg_sweeps = 1;
  o->learned = 0;
  o->coarse_amg_explicit = 2048;
  o->coarse_amg_psmooth = 1;
  o->smoother = HHO_SMOOTHER_SCHWARZ;
  o->nullspace = HHO_NULLSPACE_AUTO;
  o->vcycle_copy = HHO_COPY_CONVERT;
  o->local_build = HHO_LOCAL_AUTO;
}

int hho_mesh_create(const hho_mesh_desc *desc, hho_mesh **out) {
  ABI_BEGIN
  if (!out) hho::fail(HHO_E_INVALID_ARG, "mesh_create: out is NULL");
  *out = nullptr;
  auto m = std::make_unique<hho_mesh>();
  hho::build_mesh(desc, m.get());
  *out = m.release();
  return HHO_OK;
  ABI_END
}

void hho_mesh_destroy(hho_mesh *m) { delete m; }

int hho_problem_create(const hho_mesh *mesh, int k, int cond, int nlev, const int *degrees, const hho_options *opt,
                       hho_problem **out) {
  ABI_BEGIN
  if (!out || !mesh) hho::fail(HHO_E_INVALID_ARG, "problem_create: NULL argument");
  *out = nullptr;
  if (k < 0 || k > 6) hho::fail(HHO_E_INVALID_ARG, "problem_create: k must be in 0..6");
  if (cond != HHO_COND_V && cond != HHO_COND_VP) hho::fail(HHO_E_INVALID_ARG, "problem_create: bad condensation");
  auto P = std::make_unique<hho_problem>();
  P->mesh = mesh;
  P->k = k;
  P->cond = cond;
  P->d = mesh->dim;
  if (opt)
    P->opt = *opt;
  else
    hho_options_default(&P->opt);
  if (degrees) {
    if (nlev < 1 || degrees[0] != k) hho::fail(HHO_E_INVALID_ARG, "problem_create: degrees[0] must equal k");
    for (int i = 0; i < nlev; ++i) {
      if (degrees[i] < 0 || (i > 0 && degrees[i] >= degrees[i - 1]))
        hho::fail(HHO_E_INVALID_ARG, "problem_create: degrees must be strictly decreasing and >= 0");
      P->deg.push_back(degrees[i]);
    }
  } else {
    for (int kk = k; kk >= 0; --kk) P->deg.push_back(kk);
  }
  P->nlev = (int)P->deg.size();
  if (P->opt.restart < 1 || P->opt.restart > hho::kMaxRestartH) hho::fail(HHO_E_INVALID_ARG, "restart must be in 1..64");
  if (P->opt.coarse_restart < 1 || P->opt.coarse_restart > hho::kMaxRestartH)
    hho::fail(HHO_E_INVALID_ARG, "coarse_restart must be in 1..64");
  if (P->opt.smooth_its < 1 || P->opt.smooth_its > 2) hho::fail(HHO_E_INVALID_ARG, "smooth_its must be 1 or 2");
  if (P->opt.coarse_mode < HHO_COARSE_AUTO || P->opt.coarse_mode > HHO_COARSE_DIRECT)
    hho::fail(HHO_E_INVALID_ARG, "bad coarse_mode");
  if (P->opt.coarse_amg_sweeps < 1 || P->opt.coarse_amg_sweeps > 2)
    hho::fail(HHO_E_INVALID_ARG, "coarse_amg_sweeps must be 1 or 2");
  P->amg_nu = P->opt.coarse_amg_sweeps;
  if (P->opt.coarse_amg_explicit < 0 || P->opt.coarse_amg_explicit > hho::kAmgExplicitMax)
    hho::fail(HHO_E_INVALID_ARG, "coarse_amg_explicit must be in 0..4096");
  if (P->opt.coarse_amg_psmooth < 1 || P->opt.coarse_amg_psmooth > 2)
    hho::fail(HHO_E_INVALID_ARG, "coarse_amg_psmooth must be 1 or 2");
  if (P->opt.precision != HHO_PREC_FP64 && P->opt.precision != HHO_PREC_FP32 && P->opt.precision != HHO_PREC_BF16)
    hho::fail(HHO_E_INVALID_ARG, "bad precision");
  if (P->opt.learned != 0 && P->opt.learned != 1) hho::fail(HHO_E_INVALID_ARG, "learned must be 0 or 1");
  if (P->opt.smoother != HHO_SMOOTHER_SCHWARZ && P->opt.smoother != HHO_SMOOTHER_ILU)
    hho::fail(HHO_E_INVALID_ARG, "smoother must be HHO_SMOOTHER_SCHWARZ or HHO_SMOOTHER_ILU");
  if (P->opt.smoother == HHO_SMOOTHER_ILU && (P->opt.precision != HHO_PREC_FP64 || P->opt.learned))
    hho::fail(HHO_E_INVALID_ARG, "smoother ILU: FP64 V-cycle without the learned smoother");
  P->ilu_on = P->opt.smoother == HHO_SMOOTHER_ILU;
  if (P->opt.nullspace != HHO_NULLSPACE_AUTO && P->opt.nullspace != HHO_NULLSPACE_NONE)
    hho::fail(HHO_E_INVALID_ARG, "nullspace must be HHO_NULLSPACE_AUTO or HHO_NULLSPACE_NONE");
  if (P->opt.vcycle_copy != HHO_COPY_CONVERT && P->opt.vcycle_copy != HHO_COPY_PRODUCT)
    hho::fail(HHO_E_INVALID_ARG, "vcycle_copy must be HHO_COPY_CONVERT or HHO_COPY_PRODUCT");
  if (P->opt.vcycle_copy == HHO_COPY_PRODUCT && (P->opt.precision == HHO_PREC_FP64 || P->deg.size() < 2))
    hho::fail(HHO_E_INVALID_ARG, "vcycle_copy PRODUCT needs an FP32 or BF16 V-cycle with at least two levels");
  if (P->opt.local_build != HHO_LOCAL_AUTO && P->opt.local_build != HHO_LOCAL_HOST &&
      P->opt.local_build != HHO_LOCAL_DEVICE)
    hho::fail(HHO_E_INVALID_ARG, "local_build must be HHO_LOCAL_AUTO, HHO_LOCAL_HOST or HHO_LOCAL_DEVICE");
  if (P->opt.max_it < 1 || P->opt.coarse_max_it < 1) hho::fail(HHO_E_INVALID_ARG, "iteration limits must be >= 1");
  if (!(P->opt.rtol > 0) || !(P->opt.coarse_rtol >= 0)) hho::fail(HHO_E_INVALID_ARG, "tolerances must be > 0");
  const int d = P->d;
  // coarsest-level tolerance: the paper's 1e-3 for its iterative coarse solve in
  // 3D; in 2D, where the paper solves the coarsest level exactly, 1e-2 keeps the
  // exact solve's outer iteration count
  if (P->opt.coarse_rtol == 0) P->opt.coarse_rtol = d == 3 ? 1e-3 : 1e-2;
  {  // the patch smoother keeps a cell's face unknowns (one component for v-cond) in one wavefront's registers
    const int pk = (d == 2) ? k + 1 : (k + 1) * (k + 2) / 2;
    if (P->deg.size() > 1 && (int64_t)mesh->max_faces * (cond == 1 ? pk : d * pk) > hho::kPatchMaxRows)
      hho::fail(HHO_E_INVALID_ARG, "problem_create: a cell patch has more than 256 face unknowns per component block");
  }
  P->eta = P->opt.eta > 0 ? P->opt.eta : 4.0 * (k + 1) * (k + d) / d * mesh->max_faces;
  hho::build_topology(P.get());
  hho::init_levels(P.get());
  {
    MlpDims &md = P->md;
    const LevelInfo &L0 = P->lev[0];
    md.d = d;
    md.p = L0.p;
    md.t = L0.t;
    md.Fm = mesh->max_faces;
    md.dp = d * L0.p;
    md.n_res = 2 * (md.Fm * md.dp + md.t);
    md.n_in = md.n_res + 2 * md.Fm;
    md.n_out = md.dp + 2 * md.t;
    md.n_in16 = (md.n_in + 15) / 16 * 16;
    md.n_out16 = (md.n_out + 15) / 16 * 16;
    md.nface = L0.nface;
  }
  const int nT = hho::dim_poly(d, k), nF = hho::dim_poly(d - 1, k);
  P->lds_condense = hho::condense_lds_bytes(d, cond, nT, nF, mesh->max_faces);
  if (P->lds_condense > 64 * 1024)
    hho::fail(HHO_E_INVALID_ARG, "cell too large for the condensation kernel's LDS budget");
  *out = P.release();
  return HHO_OK;
  ABI_END
}

void hho_problem_destroy(hho_problem *p) {
  if (!p) return;
  hho::drop_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->h_st) (void)hipHostFree(p->h_st);
  delete p;
}

int hho_problem_set_data(hho_problem *p, hho_field_fn f, hho_field_fn gD, hho_field_fn gN, void *ctx) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "set_data: NULL problem");
  int qdeg = 2 * p->k + 2 + std::max(0, p->opt.quad_extra);
  p->user_rhs.clear();
  p->user_off.clear();
  p->local_dev = hho::choose_local_device(p, qdeg);
  if (p->local_dev) {
    hho::build_data_moments(p->mesh, p->k, qdeg, f, gD, gN, ctx, &p->dmom, &p->loc);
    p->cell_eta_dev = p->cell_eta.empty() ? std::vector<double>(p->mesh->nc, p->eta) : p->cell_eta;
  } else {
    hho::build_local(p->mesh, p->k, p->eta, p->cell_eta.empty() ? nullptr : p->cell_eta.data(), qdeg, f, gD, gN,
                     ctx, &p->loc);
  }
  hho::settle_auto_coarse(p);
  hho::amg_levels(p);
  p->have_data = true;
  p->setup_done = false;
  hho::Arena A;
  hho::plan(p, A);
  p->need = A.off + 256;
  return HHO_OK;
  ABI_END
}

int hho_workspace_size(const hho_problem *p, size_t *bytes) {
  ABI_BEGIN
  if (!p || !bytes) hho::fail(HHO_E_INVALID_ARG, "workspace_size: NULL argument");
  if (!p->have_data) hho::fail(HHO_E_INVALID_ARG, "workspace_size: call hho_problem_set_data first");
  *bytes = p->need;
  return HHO_OK;
  ABI_END
}

int hho_bind_workspace(hho_problem *p, void *dev_ptr, size_t bytes) {
  ABI_BEGIN
  if (!p || !dev_ptr) hho::fail(HHO_E_INVALID_ARG, "bind_workspace: NULL argument");
  if (!p->have_data) hho::fail(HHO_E_INVALID_ARG, "bind_workspace: call hho_problem_set_data first");
  if (bytes < p->need) {
    hho::set_error("bind_workspace: buffer too small");
    return HHO_E_CAPACITY;
  }
  hho::Arena A;
  A.base = (char *)(((uintptr_t)dev_ptr + 255) & ~(uintptr_t)255);
  hho::drop_graph(p);  // captured addresses change with the workspace
  hho::plan(p, A);
  p->ws = (char *)dev_ptr;
  p->ws_bytes = bytes;
  p->bound = true;
  p->setup_done = false;
  if (!p->h_st) HIPCHK(hipHostMalloc((void **)&p->h_st, sizeof(hho::GmresState)));
  return HHO_OK;
  ABI_END
}

int hho_set_graph(hho_problem *p, int enable) {
  ABI_BEGIN
  if (!p || (enable != 0 && enable != 1)) hho::fail(HHO_E_INVALID_ARG, "set_graph: bad argument");
  p->graph_on = enable == 1;
  if (!p->graph_on) hho::drop_graph(p);
  return HHO_OK;
  ABI_END
}

int hho_set_stream(hho_problem *p, void *stream) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "set_stream: NULL problem");
  p->stream = (hipStream_t)stream;
  return HHO_OK;
  ABI_END
}

int hho_setup(hho_problem *p) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "setup: NULL problem");
  if (!p->have_data) hho::fail(HHO_E_INVALID_ARG, "setup: call hho_problem_set_data first");
  if (!p->bound) hho::fail(HHO_E_INVALID_ARG, "setup: no workspace bound");
  p->setup_done = false;
  hho::device_setup(p);
  hho::set_rtol(p, p->cst, p->opt.coarse_rtol);
  p->setup_done = true;
  return HHO_OK;
  ABI_END
}

int hho_level_size(const hho_problem *p, int level, int64_t *n) {
  ABI_BEGIN
  if (!p || !n || level < 0 || level >= p->nlev) hho::fail(HHO_E_INVALID_ARG, "level_size: bad argument");
  *n = p->lev[level].N;
  return HHO_OK;
  ABI_END
}

static void need_setup(const hho_problem *p) {
  if (!p) hho::fail(HHO_E_INVALID_ARG, "NULL problem");
  if (!p->setup_done) hho::fail(HHO_E_INVALID_ARG, "call hho_setup first");
}

int hho_solve_device(hho_problem *p, double *x_dev, int *iters, double *hist, int hist_cap, double *final_rel) {
  ABI_BEGIN
  need_setup(p);
  if (p->nseg > 0) return hho::fgmres_batched(p, x_dev, iters, hist, hist_cap, final_rel);
  return hho::fgmres(p, x_dev, iters, hist, hist_cap, final_rel);
  ABI_END
}

int hho_solution_sizes(const hho_problem *p, int64_t *face_n, int64_t *p_n) {
  ABI_BEGIN
  if (!p || !face_n || !p_n) hho::fail(HHO_E_INVALID_ARG, "solution_sizes: NULL");
  const hho::LevelInfo &L0 = p->lev[0];
  *face_n = L0.nface;
  *p_n = L0.N - L0.nface;
  return HHO_OK;
  ABI_END
}

int hho_solve(hho_problem *p, double *face_out, int64_t face_cap, double *cell_p_out, int64_t p_cap, int *iters,
              double *hist, int hist_cap, double *final_rel) {
  ABI_BEGIN
  need_setup(p);
  const hho::LevelInfo &L0 = p->lev[0];
  const int64_t nfv = L0.nface, npv = L0.N - L0.nface;
  if (!face_out || !cell_p_out) hho::fail(HHO_E_INVALID_ARG, "solve: NULL output buffer");
  if (face_cap < nfv || p_cap < npv) {
    hho::set_error("solve: output buffers too small: face_cap >= " + std::to_string(nfv) + " and p_cap >= " +
                   std::to_string(npv) + " are needed");
    return HHO_E_CAPACITY;
  }
  const int rc = p->nseg > 0 ? hho::fgmres_batched(p, nullptr, iters, hist, hist_cap, final_rel)
                             : hho::fgmres(p, nullptr, iters, hist, hist_cap, final_rel);
  HIPCHK(hipMemcpyAsync(face_out, p->ox, nfv * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(cell_p_out, p->ox + nfv, npv * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return rc;
  ABI_END
}

int hho_recover_cells(hho_problem *p, const double *x_dev, double *cell_u_dev, double *cell_p_dev) {
  ABI_BEGIN
  need_setup(p);
  if (!x_dev || !cell_u_dev || !cell_p_dev) hho::fail(HHO_E_INVALID_ARG, "recover_cells: NULL pointer");
  const size_t lds = hho::recover_lds_bytes(p->d, p->loc.nT, p->loc.nF, p->max_faces);
  if (lds > 64 * 1024) hho::fail(HHO_E_INVALID_ARG, "recover_cells: cell too large for the kernel's LDS budget");
  hipStream_t s = p->stream;
  HIPCHK(hipMemsetAsync(p->err, 0, sizeof(int), s));
  hho::launch_recover(p->tp, p->cond, p->loc.nT, p->loc.nF, p->rec, p->roff, x_dev, cell_u_dev, cell_p_dev, p->err,
                      s, lds);
  HIPCHK(hipGetLastError());
  int herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, p->err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (herr) hho::fail(HHO_E_LOCAL_SINGULAR, "recover_cells: local block not SPD in cell " + std::to_string(herr - 1));
  return HHO_OK;
  ABI_END
}

int hho_get_rhs(hho_problem *p, double *b_dev) {
  ABI_BEGIN
  need_setup(p);
  if (!b_dev) hho::fail(HHO_E_INVALID_ARG, "get_rhs: NULL");
  hho::launch_copy<double>(p->lev[0].N, p->rhs, b_dev, p->stream);
  HIPCHK(hipStreamSynchronize(p->stream));
  return HHO_OK;
  ABI_END
}

int hho_get_local_cell(const hho_problem *p, int64_t cell, double *a, double *B, double *ru, double *rp, int64_t cap,
                       int64_t *nloc_out) {
  ABI_BEGIN
  if (!p || !p->have_data) hho::fail(HHO_E_INVALID_ARG, "get_local_cell: no data");
  if (cell < 0 || cell >= p->mesh->nc) hho::fail(HHO_E_INVALID_ARG, "get_local_cell: cell out of range");
  const int nloc = p->loc.nloc[cell], d = p->d, nT = p->loc.nT;
  if (nloc_out) *nloc_out = nloc;
  if (cap < (int64_t)nloc * nloc || cap < (int64_t)d * nT * nloc) {
    hho::set_error("get_local_cell: capacity too small");
    return HHO_E_CAPACITY;
  }
  std::vector<double> dev;
  const double *r;
  if (p->local_dev) {  // the record the device built (after hho_setup)
    if (!p->setup_done) hho::fail(HHO_E_INVALID_ARG, "get_local_cell: the device builds the records in hho_setup");
    dev.resize(p->loc.off[cell + 1] - p->loc.off[cell]);
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipMemcpy(dev.data(), p->rec + p->loc.off[cell], dev.size() * 8, hipMemcpyDeviceToHost));
    r = dev.data();
  } else {
    r = &p->loc.rec[p->loc.off[cell]];
  }
  if (a) std::memcpy(a, r, sizeof(double) * nloc * nloc);
  r += (int64_t)nloc * nloc;
  if (B) std::memcpy(B, r, sizeof(double) * d * nT * nloc);
  r += (int64_t)d * nT * nloc;
  if (ru) std::memcpy(ru, r, sizeof(double) * d * nloc);
  r += (int64_t)d * nloc;
  if (rp) std::memcpy(rp, r, sizeof(double) * nT);
  return HHO_OK;
  ABI_END
}

int hho_local_hp_cell(const hho_mesh *m, int k, double eta, int qdeg, int64_t cell, hho_field_fn f,
                      hho_field_fn gD, hho_field_fn gN, void *ctx, double *a, double *B, double *ru, double *rp,
                      int64_t cap, int64_t *nloc_out, int64_t *npl_out) {
  ABI_BEGIN
  if (!m) hho::fail(HHO_E_INVALID_ARG, "local_hp_cell: no mesh");
  if (k < 0 || k > 8) hho::fail(HHO_E_INVALID_ARG, "local_hp_cell: degree out of range (0..8)");
  if (!(eta > 0)) hho::fail(HHO_E_INVALID_ARG, "local_hp_cell: eta must be positive");
  if (qdeg < 2 * k + 2) hho::fail(HHO_E_INVALID_ARG, "local_hp_cell: qdeg below 2k + 2");
  if (cell < 0 || cell >= m->nc) hho::fail(HHO_E_INVALID_ARG, "local_hp_cell: cell out of range");
  hho::LocalDataHP L;
  hho::build_local_hp(m, k, eta, qdeg, f, gD, gN, ctx, &L);
  const int64_t nloc = L.nloc[cell], npl = L.npl[cell], d = L.d;
  if (nloc_out) *nloc_out = nloc;
  if (npl_out) *npl_out = npl;
  if (cap < nloc * nloc || cap < d * npl * nloc) {
    hho::set_error("local_hp_cell: capacity too small");
    return HHO_E_CAPACITY;
  }
  const double *r = &L.rec[L.off[cell]];
  if (a) std::memcpy(a, r, sizeof(double) * nloc * nloc);
  r += nloc * nloc;
  if (B) std::memcpy(B, r, sizeof(double) * d * npl * nloc);
  r += d * npl * nloc;
  if (ru) std::memcpy(ru, r, sizeof(double) * d * nloc);
  r += d * nloc;
  if (rp) std::memcpy(rp, r, sizeof(double) * npl);
  return HHO_OK;
  ABI_END
}

int hho_hp_skeleton(const hho_mesh *m, int k, double eta, int qdeg, hho_field_fn f, hho_field_fn gD, hho_field_fn gN,
                    void *ctx, int64_t *rowptr, int64_t *col, double *val, double *rhs, int64_t cap_nnz,
                    int64_t *n_out, int64_t *nnz_out) {
  ABI_BEGIN
  if (!m) hho::fail(HHO_E_INVALID_ARG, "hp_skeleton: no mesh");
  if (k < 0 || k > 8) hho::fail(HHO_E_INVALID_ARG, "hp_skeleton: degree out of range (0..8)");
  if (!(eta > 0)) hho::fail(HHO_E_INVALID_ARG, "hp_skeleton: eta must be positive");
  if (qdeg < 2 * k + 2) hho::fail(HHO_E_INVALID_ARG, "hp_skeleton: qdeg below 2k + 2");
  hho::LocalDataHP L;
  hho::build_local_hp(m, k, eta, qdeg, f, gD, gN, ctx, &L);
  std::vector<int64_t> rp, ci;
  std::vector<double> v, b;
  hho::build_skeleton_hp(m, L, rp, ci, v, b);
  const int64_t n = (int64_t)b.size(), nnz = rp.back();
  if (n_out) *n_out = n;
  if (nnz_out) *nnz_out = nnz;
  if (cap_nnz < nnz) {
    hho::set_error("hp_skeleton: capacity too small");
    return HHO_E_CAPACITY;
  }
  if (rowptr) std::memcpy(rowptr, rp.data(), sizeof(int64_t) * (n + 1));
  if (col) std::memcpy(col, ci.data(), sizeof(int64_t) * nnz);
  if (val) std::memcpy(val, v.data(), sizeof(double) * nnz);
  if (rhs) std::memcpy(rhs, b.data(), sizeof(double) * n);
  return HHO_OK;
  ABI_END
}

int hho_get_condensed_cell(hho_problem *p, int64_t cell, double *S, double *rhs, int64_t cap, int64_t *n_out) {
  ABI_BEGIN
  need_setup(p);
  if (cell < 0 || cell >= p->mesh->nc) hho::fail(HHO_E_INVALID_ARG, "get_condensed_cell: cell out of range");
  const hho::LevelInfo &L = p->lev[0];
  const int d = p->d, nfc = p->cptr[cell + 1] - p->cptr[cell];
  const int nd = nfc * d * L.p, n = nd + L.t;
  if (n_out) *n_out = n;
  if (cap < (int64_t)n * n) {
    hho::set_error("get_condensed_cell: capacity too small");
    return HHO_E_CAPACITY;
  }
  // The per-cell condensed face block lives only in the condensation staging
  // array, which the smoother setup reuses as scratch: condense again (the
  // kernel is deterministic, so every other output is rewritten unchanged; the
  // pressure part of the right-hand side goes to the outer solver's scratch).
  std::vector<double> h((size_t)n * n, 0.0), hr(n, 0.0);
  hipStream_t s = p->stream;
  const int bs = L.bs;
  const int64_t so = p->pairoff[cell] * bs * bs;
  hho::launch_condense(p->tp, p->cond, p->loc.nT, p->loc.nF, p->rec, p->roff, p->stage, L.cpl, L.spp, p->rhs_stage,
                       p->ow, p->err, s, p->lds_condense);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  std::vector<double> blk((size_t)nfc * nfc * bs * bs);
  HIPCHK(hipMemcpy(blk.data(), p->stage + so, blk.size() * 8, hipMemcpyDeviceToHost));
  const int p_ = L.p, t = L.t;
  if (p->cond == HHO_COND_V) {
    const int m = nfc * p_;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        for (int c = 0; c < d; ++c) {
          int ri = ((i / p_) * d + c) * p_ + i % p_, rj = ((j / p_) * d + c) * p_ + j % p_;
          h[(size_t)ri * n + rj] = blk[(size_t)i * m + j];
        }
  } else {
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) h[(size_t)i * n + j] = blk[(size_t)i * nd + j];
  }
  const int64_t cw = p->cond == HHO_COND_V ? (int64_t)nd * t : nd;
  std::vector<double> C(cw);
  HIPCHK(hipMemcpy(C.data(), L.cpl + (int64_t)p->cptr[cell] * d * p_ * (p->cond == HHO_COND_V ? t : 1), cw * 8,
                   hipMemcpyDeviceToHost));
  for (int i = 0; i < nd; ++i)
    for (int q = 0; q < t; ++q) {
      double v = p->cond == HHO_COND_V ? C[(size_t)i * t + q] : C[i];
      h[(size_t)i * n + nd + q] = v;
      h[(size_t)(nd + q) * n + i] = v;
    }
  if (p->cond == HHO_COND_V) {
    std::vector<double> Pp((size_t)t * t);
    HIPCHK(hipMemcpy(Pp.data(), L.spp + (int64_t)cell * t * t, Pp.size() * 8, hipMemcpyDeviceToHost));
    for (int q = 0; q < t; ++q)
      for (int q2 = 0; q2 < t; ++q2) h[(size_t)(nd + q) * n + nd + q2] = Pp[(size_t)q * t + q2];
  }
  HIPCHK(hipMemcpy(hr.data(), p->rhs_stage + (int64_t)p->cptr[cell] * d * p_, nd * 8, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(hr.data() + nd, p->ow + (int64_t)cell * t, t * 8, hipMemcpyDeviceToHost));
  if (S) std::memcpy(S, h.data(), h.size() * 8);
  if (rhs) std::memcpy(rhs, hr.data(), hr.size() * 8);
  return HHO_OK;
  ABI_END
}

int hho_level_apply(hho_problem *p, int level, const double *x, double *y) {
  ABI_BEGIN
  need_setup(p);
  if (level < 0 || level >= p->nlev || !x || !y) hho::fail(HHO_E_INVALID_ARG, "level_apply: bad argument");
  hho::launch_spmv<double>(p->tp, hho::dlev64(p, level), x, nullptr, nullptr, y, p->stream);
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_vcycle_level_apply(hho_problem *p, int level, int which, const double *x, double *y) {
  ABI_BEGIN
  need_setup(p);
  if (level < 0 || level >= p->nlev || !x || !y || (which != 0 && which != 1))
    hho::fail(HHO_E_INVALID_ARG, "vcycle_level_apply: bad argument");
  const hho::LevelInfo &L = p->lev[level];
  if (which == 1 && !L.sinv) hho::fail(HHO_E_INVALID_ARG, "vcycle_level_apply: this level has no smoother");
  hipStream_t s = p->stream;
  const bool mixed = p->opt.precision != HHO_PREC_FP64 && level < p->nlev - 1;
  if (!mixed) {
    if (which == 0) {
      hho::launch_spmv<double>(p->tp, hho::dlev64(p, level), x, nullptr, nullptr, y, s);
    } else {
      double *zs1 = p->ow;
      hho::launch_precond<double>(p->tp, hho::dlev64(p, level), x, nullptr, nullptr, y, zs1, p->max_faces, s);
      hho::launch_combine<double>(L.nface, zs1, y, s);
    }
  } else {
    // the level's own FP32 V-cycle vectors serve as input and output
    const hho::VBufs<float> &V = p->lev[level].v32;
    hho::launch_convert<float, double>(x, V.z1, L.N, s);
    const bool b16 = p->opt.precision == HHO_PREC_BF16;
    if (which == 0) {
      if (b16)
        hho::launch_spmv<float>(p->tp, hho::dlev16(p, level), V.z1, nullptr, nullptr, V.w1, s);
      else
        hho::launch_spmv<float>(p->tp, hho::dlev32(p, level), V.z1, nullptr, nullptr, V.w1, s);
    } else {
      if (b16)
        hho::launch_precond<float>(p->tp, hho::dlev16(p, level), V.z1, nullptr, nullptr, V.w1, V.zs1, p->max_faces, s);
      else
        hho::launch_precond<float>(p->tp, hho::dlev32(p, level), V.z1, nullptr, nullptr, V.w1, V.zs1, p->max_faces, s);
      hho::launch_combine<float>(L.nface, V.zs1, V.w1, s);
    }
    hho::launch_convert<double, float>(V.w1, y, L.N, s);
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_precond_apply(hho_problem *p, int level, const double *r, double *z) {
  ABI_BEGIN
  need_setup(p);
  if (level < 0 || level >= p->nlev || !r || !z) hho::fail(HHO_E_INVALID_ARG, "precond_apply: bad argument");
  const hho::LevelInfo &L = p->lev[level];
  if (p->ilu_on) {
    if (!hho::ilu_level(p, level)) hho::fail(HHO_E_INVALID_ARG, "precond_apply: this level has no smoother");
    hho::ilu_apply(p, level, r, z);
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipGetLastError());
    return HHO_OK;
  }
  if (!L.sinv) hho::fail(HHO_E_INVALID_ARG, "precond_apply: this level has no smoother (dense coarse level)");
  double *zs1 = p->ow;  // level-0 length covers the face part of every level
  hho::launch_precond<double>(p->tp, hho::dlev64(p, level), r, nullptr, nullptr, z, zs1, p->max_faces, p->stream);
  hho::launch_combine<double>(L.nface, zs1, z, p->stream);
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_vcycle_apply(hho_problem *p, const double *b, double *x) {
  ABI_BEGIN
  need_setup(p);
  if (!b || !x) hho::fail(HHO_E_INVALID_ARG, "vcycle_apply: NULL");
  hho::apply_vcycle(p, b, x);
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_debug_copy(hho_problem *p, const char *name, int level, double *out, int64_t cap, int64_t *n_out) {
  ABI_BEGIN
  need_setup(p);
  std::string nm = name ? name : "";
  const double *src = nullptr;
  int64_t n = 0;
  if (nm.rfind("amg_", 0) == 0) {
    if (!p->coarse_amg || level < 0 || level >= p->amgd.nlev) hho::fail(HHO_E_INVALID_ARG, "debug_copy: bad AMG level");
    const hho::AmgDevLevel &G = p->amgd.lev[level];
    if (nm == "amg_val") src = G.val, n = G.nnz;
    else if (nm == "amg_pval") src = G.pval, n = G.npe;
    else if (nm == "amg_dinv") src = G.dinv, n = G.n;
    else if (nm == "amg_lam") src = G.lam, n = 1;
    else if (nm == "amg_ainv") src = p->amgd.ainv, n = (int64_t)G.n * G.n;
  } else if (nm == "sd" && p->coarse_amg) {
    src = p->Sd, n = p->mesh->nc;
  }
  if (!src) hho::fail(HHO_E_INVALID_ARG, "debug_copy: unknown array " + nm);
  if (n_out) *n_out = n;
  if (cap < n) {
    hho::set_error("debug_copy: capacity");
    return HHO_E_CAPACITY;
  }
  HIPCHK(hipMemcpy(out, src, n * 8, hipMemcpyDeviceToHost));
  return HHO_OK;
  ABI_END
}

int hho_coarse_prec_apply(hho_problem *p, const double *v, double *z) {
  ABI_BEGIN
  need_setup(p);
  if (!v || !z) hho::fail(HHO_E_INVALID_ARG, "coarse_prec_apply: NULL");
  if (!p->coarse_amg) hho::fail(HHO_E_INVALID_ARG, "coarse_prec_apply: the coarsest level does not use the AMG solver");
  const hho::LevelInfo &L = p->lev[p->nlev - 1];
  hho::bp_apply(p->tp, p->amgd, L.nface, L.cpl, p->Sd, v, z, p->amg_nu, p->stream);
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_coarse_solve_apply(hho_problem *p, const double *b, double *x) {
  ABI_BEGIN
  need_setup(p);
  if (!b || !x) hho::fail(HHO_E_INVALID_ARG, "coarse_solve_apply: NULL");
  hho::LevelInfo &L = p->lev[p->nlev - 1];
  HIPCHK(hipMemcpyAsync(L.v64.b, b, L.N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  p->coarse_its = 0;
  hho::coarse_solve(p);
  HIPCHK(hipMemcpyAsync(x, L.v64.w, L.N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_direct_info(const hho_problem *p, const char *name, int64_t *out, int64_t cap, int64_t *n_out) {
  ABI_BEGIN
  if (!p || !name || !n_out) hho::fail(HHO_E_INVALID_ARG, "direct_info: NULL");
  if (!p->coarse_direct || p->nd.m.empty())
    hho::fail(HHO_E_INVALID_ARG, "direct_info: the problem has no sparse direct coarse solver (or no data yet)");
  const hho::NdHost &H = p->nd;
  const std::string n(name);
  std::vector<int64_t> v;
  auto put = [&](const auto &src) { v.assign(src.begin(), src.end()); };
  if (n == "m") put(H.m);
  else if (n == "nfs") put(H.nfs);
  else if (n == "child") put(H.child);
  else if (n == "dofoff") put(H.dofoff);
  else if (n == "dof") put(H.dof);
  else if (n == "cmap") put(H.cmap);
  else if (n == "hptr") put(H.hptr);
  else if (n == "hfront") put(H.hfront);
  else if (n == "pinned") put(H.pins);
  else if (n == "sizes") v = {H.nfront, H.nheight, H.total, H.factor_entries, H.maxm};
  else if (n == "hfwd" || n == "hbwd") {
    for (int h = 0; h < H.nheight; ++h) {
      int64_t ent = 0, unk = 0;
      for (int32_t x = H.hptr[h]; x < H.hptr[h + 1]; ++x) {
        const int64_t m = H.m[H.hfront[x]], f = H.nfs[H.hfront[x]];
        ent += n == "hfwd" ? (m - f) * f : f * m;
        unk += m;
      }
      v.push_back(ent);
      v.push_back(unk);
    }
  }
  else hho::fail(HHO_E_INVALID_ARG, "direct_info: unknown name " + n);
  *n_out = (int64_t)v.size();
  if ((int64_t)v.size() > cap) hho::fail(HHO_E_CAPACITY, "direct_info: buffer too small");
  if (out) std::copy(v.begin(), v.end(), out);
  return HHO_OK;
  ABI_END
}

int hho_upload(hho_problem *p) {
  ABI_BEGIN
  if (!p || !p->have_data || !p->bound) hho::fail(HHO_E_INVALID_ARG, "upload: needs data and a bound workspace");
  hho::device_upload(p);
  return HHO_OK;
  ABI_END
}

static double time_kernel_ms(hho_problem *p, int kind, int level, int reps) {
  if (level < 0 || level >= p->nlev || reps < 1) hho::fail(HHO_E_INVALID_ARG, "time_kernel: bad argument");
  hipStream_t s = p->stream;
  const hho::LevelInfo &L = p->lev[level];
  const bool mixed = p->opt.precision != HHO_PREC_FP64 && level < p->nlev - 1;
  const bool b16 = p->opt.precision == HHO_PREC_BF16;
  if ((kind == 1 || kind == 2) && !L.sinv) hho::fail(HHO_E_INVALID_ARG, "time_kernel: level has no smoother");
  // inputs: the level's operator applied to the outer solver's scratch vectors
  hho::launch_fill<double>(L.N, 1.0, p->ox, s);
  auto one = [&]() {
    switch (kind) {
      case 0:
        hho::launch_spmv<double>(p->tp, hho::dlev64(p, level), p->ox, nullptr, nullptr, p->ow, s);
        break;
      case 1:
        hho::launch_precond<double>(p->tp, hho::dlev64(p, level), p->ox, nullptr, nullptr, p->ow, p->or_,
                                    p->max_faces, s);
        break;
      case 2:
        if (mixed) {
          const hho::VBufs<float> &V = p->lev[level].v32;
          if (b16)
            hho::launch_spmv<float>(p->tp, hho::dlev16(p, level), V.zs0, V.zs1, V.z1, V.w1, s);
          else
            hho::launch_spmv<float>(p->tp, hho::dlev32(p, level), V.zs0, V.zs1, V.z1, V.w1, s);
        } else {
          const hho::VBufs<double> &V = p->lev[level].v64;
          hho::launch_spmv<double>(p->tp, hho::dlev64(p, level), V.zs0, V.zs1, V.z1, V.w1, s);
        }
        break;
      case 3:
        hho::apply_vcycle(p, p->ox, p->ow);
        break;
      default:
        hho::fail(HHO_E_INVALID_ARG, "time_kernel: unknown kind");
    }
  };
  if (kind == 2) {  // defined inputs for the split operator
    if (mixed) {
      hho::launch_fill<float>(L.N, 1.0f, p->lev[level].v32.zs0, s);
      hho::launch_fill<float>(L.nface, 0.0f, p->lev[level].v32.zs1, s);
    } else {
      hho::launch_fill<double>(L.N, 1.0, p->lev[level].v64.zs0, s);
      hho::launch_fill<double>(L.nface, 0.0, p->lev[level].v64.zs1, s);
    }
  }
  one();
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  HIPCHK(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i) one();
  HIPCHK(hipEventRecord(b, s));
  HIPCHK(hipEventSynchronize(b));
  float ms;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  HIPCHK(hipEventDestroy(a));
  HIPCHK(hipEventDestroy(b));
  HIPCHK(hipGetLastError());
  return ms / reps;
}

int hho_time_kernel(hho_problem *p, int kind, int level, int reps, double *avg_ms) {
  ABI_BEGIN
  need_setup(p);
  if (!avg_ms) hho::fail(HHO_E_INVALID_ARG, "time_kernel: bad argument");
  *avg_ms = time_kernel_ms(p, kind, level, reps);
  return HHO_OK;
  ABI_END
}

// Autotuner: the fastest launch shape of each level's operator kernel and patch
// factorisation, measured on the problem's own data.
int hho_autotune(hho_problem *p, int reps, int *choices) {
  ABI_BEGIN
  need_setup(p);
  if (reps < 1) hho::fail(HHO_E_INVALID_ARG, "autotune: reps must be >= 1");
  hipStream_t s = p->stream;
  for (int l = 0; l < p->nlev; ++l) {
    hho::LevelInfo &L = p->lev[l];
    const int kind = L.sinv ? 2 : 0;
    double best = 1e300;
    int pick = 0;
    for (int bs : {64, 128, 256}) {
      L.spmv_block = bs;
      const double ms = time_kernel_ms(p, kind, l, reps);
      if (ms < best) best = ms, pick = bs;
    }
    L.spmv_block = pick;
    int pick_patch = 0;
    if (L.sinv) {
      best = 1e300;
      hipEvent_t a, b;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      for (int th : {0, 64, 128, 256, 512}) {  // 0: register sweep where it applies
        const size_t lds = hho::patch_lds_bytes(p->d, p->cond, L.p, L.t, p->max_faces);
        HIPCHK(hipEventRecord(a, s));
        hho::launch_patch_setup(p->tp, p->cond, L.p, L.t, L.bsr, L.cpl, L.spp, L.sinv, L.xinv, L.sig, p->stage,
                                p->err + 1, s, lds, th);
        HIPCHK(hipEventRecord(b, s));
        HIPCHK(hipEventSynchronize(b));
        float ms;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        if (ms < best) best = ms, pick_patch = th;
      }
      HIPCHK(hipEventDestroy(a));
      HIPCHK(hipEventDestroy(b));
      L.patch_threads = pick_patch;
    }
    if (choices) {
      choices[2 * l] = pick;
      choices[2 * l + 1] = pick_patch;
    }
  }
  p->setup_done = false;  // factors were recomputed while timing: run hho_setup again
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_set_tolerances(hho_problem *p, double rtol, int max_it, double coarse_rtol, int coarse_max_it) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "set_tolerances: NULL problem");
  if (!(rtol > 0 && rtol < 1) || max_it < 1 || !(coarse_rtol > 0 && coarse_rtol < 1) || coarse_max_it < 1)
    hho::fail(HHO_E_INVALID_ARG, "set_tolerances: need 0 < rtol, coarse_rtol < 1 and positive iteration limits");
  p->opt.rtol = rtol;
  p->opt.max_it = max_it;
  p->opt.coarse_rtol = coarse_rtol;
  p->opt.coarse_max_it = coarse_max_it;
  return HHO_OK;
  ABI_END
}

int hho_probe_arm(hho_problem *p, unsigned mask, int stride) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "probe_arm: NULL problem");
  if (mask & ~(unsigned)HHO_PROBE_ALL) hho::fail(HHO_E_INVALID_ARG, "probe_arm: unknown class bit");
  if (stride < 1) hho::fail(HHO_E_INVALID_ARG, "probe_arm: stride must be >= 1");
  if (p->bound) HIPCHK(hipStreamSynchronize(p->stream));
  p->probe.mask = mask;
  p->probe.stride = stride;
  p->probe.reset();
  return HHO_OK;
  ABI_END
}

int hho_probe_read(hho_problem *p, int kind, int level, int64_t *timed, double *total_ms, int64_t *launches) {
  ABI_BEGIN
  if (!p || !timed || !total_ms) hho::fail(HHO_E_INVALID_ARG, "probe_read: NULL");
  const int ci = hho::KernelProbe::class_index(kind);
  if (ci >= hho::kProbeClasses || (kind & (kind - 1))) hho::fail(HHO_E_INVALID_ARG, "probe_read: kind must be one class bit");
  if (level >= hho::kProbeLevels) hho::fail(HHO_E_INVALID_ARG, "probe_read: level out of range");
  if (p->bound) HIPCHK(hipStreamSynchronize(p->stream));
  if (p->probe.failed) hho::fail(HHO_E_DEVICE, "probe_read: an event could not be created or recorded");
  int64_t cnt = 0;
  double ms = 0;
  for (const hho::KernelProbe::Rec &r : p->probe.recs) {
    if (r.kind != kind || (level >= 0 && r.level != level)) continue;
    float t;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++cnt;
  }
  *timed = cnt;
  *total_ms = ms;
  if (launches) {
    int64_t all = 0;
    for (int l = 0; l < hho::kProbeLevels; ++l)
      if (level < 0 || l == level) all += p->probe.seen[ci][l];
    *launches = all;
  }
  return HHO_OK;
  ABI_END
}

int hho_probe_clear(hho_problem *p) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "probe_clear: NULL");
  if (p->bound) HIPCHK(hipStreamSynchronize(p->stream));
  p->probe.reset();
  return HHO_OK;
  ABI_END
}

int hho_amg_level_info(const hho_problem *p, int level, int64_t *info) {
  ABI_BEGIN
  if (!p || !info) hho::fail(HHO_E_INVALID_ARG, "amg_level_info: NULL");
  if (!p->coarse_amg || level < 0 || level >= (int)p->amgh.levels.size())
    hho::fail(HHO_E_INVALID_ARG, "amg_level_info: no such AMG level");
  const hho::AmgHostLevel &H = p->amgh.levels[level];
  info[0] = H.n;
  info[1] = H.nc;
  info[2] = (int64_t)H.ci.size();
  info[3] = (int64_t)H.pci.size();
  info[4] = (int64_t)H.bci.size();
  info[5] = (int64_t)p->amgd.expl;
  info[6] = (int64_t)p->amgh.levels.size();
  return HHO_OK;
  ABI_END
}

int hho_get_timings(const hho_problem *p, double *t, int n) {
  ABI_BEGIN
  if (!p || !t) hho::fail(HHO_E_INVALID_ARG, "get_timings: NULL");
  for (int i = 0; i < n && i < 16; ++i) t[i] = p->timings[i];
  return HHO_OK;
  ABI_END
}

}  // extern "C"

// ------------------------------------------------------------ learned fine-level smoother
static void need_learned(const hho_problem *p) {
  if (!p) hho::fail(HHO_E_INVALID_ARG, "learned: NULL problem");
  if (!p->opt.learned) hho::fail(HHO_E_INVALID_ARG, "learned: create the problem with options.learned = 1");
  if (!p->bound) hho::fail(HHO_E_INVALID_ARG, "learned: bind a workspace first");
}

int hho_learned_dims(const hho_problem *p, int *n_in, int *n_out, int *hidden, int64_t *n_params) {
  ABI_BEGIN
  if (!p) hho::fail(HHO_E_INVALID_ARG, "learned_dims: NULL problem");
  if (n_in) *n_in = p->md.n_in;
  if (n_out) *n_out = p->md.n_out;
  if (hidden) *hidden = hho::kMlpHidden;
  if (n_params) *n_params = hho::mlp_param_count(p->md);
  return HHO_OK;
  ABI_END
}

int hho_learned_set_params(hho_problem *p, const float *prm, int64_t n) {
  ABI_BEGIN
  need_learned(p);
  const int64_t np = hho::mlp_param_count(p->md);
  if (!prm || n != np) hho::fail(HHO_E_INVALID_ARG, "learned_set_params: need exactly n_params values");
  HIPCHK(hipMemcpyAsync(p->mlp_prm, prm, np * sizeof(float), hipMemcpyHostToDevice, p->stream));
  hho::launch_mlp_pack(p->md, p->mlp_prm, p->mlp_w1b, p->mlp_w2b, p->stream);
  hho::launch_fill<float>(np, 0.0f, p->mlp_m, p->stream);
  hho::launch_fill<float>(np, 0.0f, p->mlp_v, p->stream);
  HIPCHK(hipStreamSynchronize(p->stream));
  p->adam_step = 0;
  p->learned_ready = true;
  return HHO_OK;
  ABI_END
}

int hho_learned_get_params(const hho_problem *p, float *prm, int64_t n) {
  ABI_BEGIN
  need_learned(p);
  const int64_t np = hho::mlp_param_count(p->md);
  if (!prm || n != np) hho::fail(HHO_E_INVALID_ARG, "learned_get_params: need exactly n_params values");
  if (!p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_get_params: no parameters set");
  HIPCHK(hipMemcpyAsync(prm, p->mlp_prm, np * sizeof(float), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return HHO_OK;
  ABI_END
}

int hho_learned_enable(hho_problem *p, int on) {
  ABI_BEGIN
  need_learned(p);
  if (on && !p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_enable: set or train parameters first");
  p->learned_on = on != 0;
  return HHO_OK;
  ABI_END
}

int hho_learned_apply(hho_problem *p, const double *r, double *z) {
  ABI_BEGIN
  need_learned(p);
  need_setup(p);
  if (!p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_apply: no parameters set");
  if (!r || !z) hho::fail(HHO_E_INVALID_ARG, "learned_apply: NULL");
  const hho::MlpDims &md = p->md;
  hipStream_t s = p->stream;
  hho::launch_mlp_windows<double>(p->tp, md, r, p->mlp_X, p->mlp_sc, s);
  hho::launch_mlp_forward(p->tp.nf, md, p->mlp_X, nullptr, p->mlp_prm, p->mlp_w1b, p->mlp_w2b, nullptr, p->mlp_Y, s);
  hho::launch_mlp_scatter<double>(p->tp, md, p->lev[0].N, p->mlp_Y, p->mlp_sc, z, s);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

int hho_learned_collect(hho_problem *p, const double *x_true, int cycles, float *X, float *Tg, int64_t cap,
                        int64_t *n_out) {
  ABI_BEGIN
  need_learned(p);
  need_setup(p);
  if (!x_true || !X || !Tg || !n_out || cycles < 1) hho::fail(HHO_E_INVALID_ARG, "learned_collect: bad argument");
  const hho::MlpDims &md = p->md;
  const int64_t nf = p->tp.nf, need = (int64_t)cycles * nf;
  if (cap < need) {
    *n_out = need;
    hho::set_error("learned_collect: capacity below cycles * n_faces samples");
    return HHO_E_CAPACITY;
  }
  hipStream_t s = p->stream;
  const hho::DLevel<double> D = hho::dlev64(p, 0);
  const int64_t n = D.N;
  const bool was_on = p->learned_on;
  p->learned_on = false;  // pairs come from the plain V-cycle
  hho::launch_spmv<double>(p->tp, D, x_true, nullptr, nullptr, p->ob, s);  // b = S x_true
  hho::launch_fill<double>(n, 0.0, p->ox, s);
  hho::launch_fill<double>(2, 1.0, p->scal + 2, s);  // ratio 1/1 for the update below
  for (int c = 0; c < cycles; ++c) {
    hho::launch_residual<double>(p->tp, D, p->ob, p->ox, p->or_, s);
    float *Xc = X + (int64_t)c * nf * md.n_in;
    hho::launch_mlp_windows<double>(p->tp, md, p->or_, Xc, p->mlp_sc, s);
    hho::launch_mlp_targets(p->tp, md, x_true, p->ox, p->mlp_sc, Tg + (int64_t)c * nf * md.n_out, s);
    if (c + 1 < cycles) {
      hho::apply_vcycle(p, p->or_, p->ow);
      hho::launch_axpy_ratio<double>(n, p->scal + 2, 1.0, p->ow, p->ox, s);  // x += V(r)
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  p->learned_on = was_on;
  *n_out = need;
  return HHO_OK;
  ABI_END
}

// work arrays of one loss-and-gradient evaluation over at most kMlpMaxBatch rows
struct MlpWork {
  float *Z, *Y, *dY, *dZ, *g;  // hidden activations, outputs, their gradients, parameter gradient
  double *partial;             // per-block partial sums of the squared errors
};

static MlpWork mlp_work(hho_problem *p) {
  return {p->mlp_Z, p->mlp_Yb, p->mlp_dY, p->mlp_dZ, p->mlp_g, p->partial};
}

// loss and gradient (into w.g) of the batch rows (rows == null: rows 0..B-1) at the
// current parameters; the summed squared error goes to loss_dev
static double mlp_loss_grad(hho_problem *p, const MlpWork &w, const float *X, const float *Tg, const int *rows, int B,
                            double *loss_dev) {
  const hho::MlpDims &md = p->md;
  hipStream_t s = p->stream;
  hho::launch_mlp_forward(B, md, X, rows, p->mlp_prm, p->mlp_w1b, p->mlp_w2b, w.Z, w.Y, s);
  const int G = hho::launch_mlp_backward(B, md.n_in, md.n_out, X, rows, Tg, p->mlp_w2b, w.Z, w.Y, w.dY, w.dZ, w.g,
                                         w.partial, s);
  hho::launch_sum_finish(G, w.partial, loss_dev, s);
  return 0.5 / B;  // factor turning the summed squares into the loss
}

int hho_learned_grad(hho_problem *p, const float *X, const float *Tg, int64_t n, float *grad, double *loss) {
  ABI_BEGIN
  need_learned(p);
  if (!p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_grad: no parameters set");
  if (!X || !Tg || !grad || !loss || n < 1 || n > hho::kMlpMaxBatch)
    hho::fail(HHO_E_INVALID_ARG, "learned_grad: bad argument (1 <= n <= 4096)");
  const double f = mlp_loss_grad(p, mlp_work(p), X, Tg, nullptr, (int)n, p->mlp_loss);
  const int64_t np = hho::mlp_param_count(p->md);
  double ls = 0;
  HIPCHK(hipMemcpyAsync(grad, p->mlp_g, np * sizeof(float), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(&ls, p->mlp_loss, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  *loss = f * ls;
  return HHO_OK;
  ABI_END
}

// ------------------------------------------------------------ allocation-free gradient
// hho_learned_grad_noalloc keeps its work arrays in this file-scope device array
// instead of the problem's workspace: hidden activations and their gradients
// (kMlpMaxBatch x kMlpHidden floats each), outputs and their gradients
// (kMlpMaxBatch x kNoallocMaxOut floats each), the parameter gradient
// (kNoallocMaxParams floats), the per-block loss partials and the summed loss.
// Every array is written before it is read within one call, so nothing is
// cleared.  Each device holds its own copy; host code reaches it only through
// the address hipGetSymbolAddress returns on that device.
namespace hho {
constexpr int64_t kNoallocMaxOut = 256;
constexpr int64_t kNoallocMaxParams = int64_t(1) << 20;
constexpr int64_t kNoallocPartials = 512;
constexpr int64_t kNoallocZ = (int64_t)kMlpMaxBatch * kMlpHidden * sizeof(float);
constexpr int64_t kNoallocY = (int64_t)kMlpMaxBatch * kNoallocMaxOut * sizeof(float);
constexpr int64_t kNoallocG = kNoallocMaxParams * sizeof(float);
constexpr int64_t kNoallocBytes = 2 * kNoallocZ + 2 * kNoallocY + kNoallocG + (kNoallocPartials + 256) * sizeof(double);
constexpr int kNoallocMaxDevices = 64;
}  // namespace hho

static __device__ __align__(256) unsigned char scratch[hho::kNoallocBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[hho::kNoallocMaxDevices];

// device address of `scratch` on the current device, looked up once per device
static char *noalloc_scratch(hho_problem *p) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= hho::kNoallocMaxDevices) hho::fail(HHO_E_DEVICE, "learned_grad_noalloc: device ordinal out of range");
  hipPointerAttribute_t attr{};
  HIPCHK(hipPointerGetAttributes(&attr, p->ws));
  if (attr.device != dev)
    hho::fail(HHO_E_INVALID_ARG, "learned_grad_noalloc: make the device of the problem's workspace current first");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) hho::fail(HHO_E_DEVICE, "learned_grad_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return (char *)g_scratch_ptr[dev];
}

int hho_learned_grad_noalloc(hho_problem *p, const float *X, const float *Tg, int64_t n, float *grad, double *loss) {
  ABI_BEGIN
  need_learned(p);
  if (!p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_grad_noalloc: no parameters set");
  if (!X || !Tg || !grad || !loss || n < 1) hho::fail(HHO_E_INVALID_ARG, "learned_grad_noalloc: bad argument");
  const hho::MlpDims &md = p->md;
  const int64_t np = hho::mlp_param_count(md);
  if (n > hho::kMlpMaxBatch || md.n_out > hho::kNoallocMaxOut || np > hho::kNoallocMaxParams) {
    hho::set_error("learned_grad_noalloc: beyond the scratch limits (rows <= " + std::to_string(hho::kMlpMaxBatch) +
                   ", outputs <= " + std::to_string(hho::kNoallocMaxOut) + ", parameters <= " +
                   std::to_string(hho::kNoallocMaxParams) + ")");
    return HHO_E_CAPACITY;
  }
  char *base = noalloc_scratch(p);
  MlpWork w;
  w.Z = (float *)base;
  w.dZ = (float *)(base + hho::kNoallocZ);
  w.Y = (float *)(base + 2 * hho::kNoallocZ);
  w.dY = (float *)(base + 2 * hho::kNoallocZ + hho::kNoallocY);
  w.g = (float *)(base + 2 * hho::kNoallocZ + 2 * hho::kNoallocY);
  w.partial = (double *)(base + 2 * hho::kNoallocZ + 2 * hho::kNoallocY + hho::kNoallocG);
  double *ls_dev = w.partial + hho::kNoallocPartials;
  const double f = mlp_loss_grad(p, w, X, Tg, nullptr, (int)n, ls_dev);
  double ls = 0;
  HIPCHK(hipMemcpyAsync(grad, w.g, np * sizeof(float), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(&ls, ls_dev, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  HIPCHK(hipGetLastError());
  *loss = f * ls;
  return HHO_OK;
  ABI_END
}

int hho_learned_train(hho_problem *p, const float *X, const float *Tg, int64_t n, int steps, int batch, float lr,
                      uint64_t seed, float *loss_hist) {
  ABI_BEGIN
  need_learned(p);
  if (!p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_train: set initial parameters first");
  if (!X || !Tg || n < 1 || steps < 1 || steps > hho::kMlpMaxSteps || batch < 1 || batch > hho::kMlpMaxBatch ||
      !(lr > 0))
    hho::fail(HHO_E_INVALID_ARG, "learned_train: bad argument");
  hipStream_t s = p->stream;
  const int64_t np = hho::mlp_param_count(p->md);
  double f = 0;
  for (int it = 0; it < steps; ++it) {
    hho::launch_mlp_rows(batch, n, seed, p->adam_step, p->mlp_rows, s);
    f = mlp_loss_grad(p, mlp_work(p), X, Tg, p->mlp_rows, batch, p->mlp_loss + it);
    hho::launch_mlp_adam(np, p->mlp_prm, p->mlp_g, p->mlp_m, p->mlp_v, lr, ++p->adam_step, s);
    hho::launch_mlp_pack(p->md, p->mlp_prm, p->mlp_w1b, p->mlp_w2b, s);
  }
  if (loss_hist) {
    std::vector<double> tmp(steps);
    HIPCHK(hipMemcpyAsync(tmp.data(), p->mlp_loss, steps * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < steps; ++i) loss_hist[i] = (float)(f * tmp[i]);
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  return HHO_OK;
  ABI_END
}

// ------------------------------------------------------------ batches of problems
// disjoint union of n mesh descriptors (member i's faces and cells follow those
// of members 0..i-1); face_offsets / cell_offsets (may be null) get n+1 entries
static void build_union_mesh(const hho_mesh_desc *descs, int n, hho_mesh *m, int64_t *face_offsets,
                             int64_t *cell_offsets) {
  const int dim = descs[0].dim;
  std::vector<double> verts;
  std::vector<int64_t> fptr(1, 0), fvtx, cptr(1, 0), cface;
  std::vector<int8_t> fbc;
  int64_t nv = 0, nf = 0, nc = 0;
  for (int i = 0; i < n; ++i) {
    const hho_mesh_desc &d = descs[i];
    if (d.dim != dim) hho::fail(HHO_E_INVALID_ARG, "mesh union: meshes of different dimensions");
    if (!d.verts || !d.face_ptr || !d.face_vtx || !d.cell_ptr || !d.cell_face || !d.face_bc || d.n_faces <= 0 ||
        d.n_cells <= 0 || d.n_verts <= 0)
      hho::fail(HHO_E_INVALID_ARG, "mesh union: empty or NULL member mesh");
    if (face_offsets) face_offsets[i] = nf;
    if (cell_offsets) cell_offsets[i] = nc;
    verts.insert(verts.end(), d.verts, d.verts + d.n_verts * dim);
    for (int64_t f = 0; f < d.n_faces; ++f) {
      for (int64_t e = d.face_ptr[f]; e < d.face_ptr[f + 1]; ++e) fvtx.push_back(d.face_vtx[e] + nv);
      fptr.push_back((int64_t)fvtx.size());
    }
    for (int64_t c = 0; c < d.n_cells; ++c) {
      for (int64_t e = d.cell_ptr[c]; e < d.cell_ptr[c + 1]; ++e) cface.push_back(d.cell_face[e] + nf);
      cptr.push_back((int64_t)cface.size());
    }
    fbc.insert(fbc.end(), d.face_bc, d.face_bc + d.n_faces);
    nv += d.n_verts;
    nf += d.n_faces;
    nc += d.n_cells;
  }
  if (face_offsets) face_offsets[n] = nf;
  if (cell_offsets) cell_offsets[n] = nc;
  hho_mesh_desc u{dim, nv, verts.data(), nf, fptr.data(), fvtx.data(), nc, cptr.data(), cface.data(), fbc.data()};
  hho::build_mesh(&u, m);
}

int hho_mesh_create_union(const hho_mesh_desc *descs, int n, hho_mesh **out, int64_t *face_offsets,
                          int64_t *cell_offsets) {
  ABI_BEGIN
  if (!descs || n < 1 || !out) hho::fail(HHO_E_INVALID_ARG, "mesh_create_union: bad argument");
  *out = nullptr;
  auto m = std::make_unique<hho_mesh>();
  build_union_mesh(descs, n, m.get(), face_offsets, cell_offsets);
  *out = m.release();
  return HHO_OK;
  ABI_END
}

int hho_problem_set_segments(hho_problem *p, int n, const int64_t *face_ptr, const int64_t *cell_ptr) {
  ABI_BEGIN
  if (!p || n < 1 || !face_ptr || !cell_ptr) hho::fail(HHO_E_INVALID_ARG, "set_segments: bad argument");
  if (p->have_data) hho::fail(HHO_E_INVALID_ARG, "set_segments: call before hho_problem_set_data");
  const hho_mesh *m = p->mesh;
  if (face_ptr[0] != 0 || cell_ptr[0] != 0 || face_ptr[n] != m->nf || cell_ptr[n] != m->nc)
    hho::fail(HHO_E_INVALID_ARG, "set_segments: ranges must partition the faces and the cells");
  std::vector<int32_t> fseg(m->nf, -1);
  for (int i = 0; i < n; ++i) {
    if (face_ptr[i + 1] <= face_ptr[i] || cell_ptr[i + 1] <= cell_ptr[i])
      hho::fail(HHO_E_INVALID_ARG, "set_segments: empty or decreasing range");
    for (int64_t f = face_ptr[i]; f < face_ptr[i + 1]; ++f) fseg[f] = i;
  }
  for (int i = 0; i < n; ++i)
    for (int64_t c = cell_ptr[i]; c < cell_ptr[i + 1]; ++c)
      for (int64_t e = m->cptr[c]; e < m->cptr[c + 1]; ++e)
        if (fseg[m->cface[e]] != i) hho::fail(HHO_E_INVALID_ARG, "set_segments: a cell and its faces lie in different segments");
  // every member is the problem it would be alone: mixed boundary types would give
  // some members a pressure null space and others none, which one border cannot
  // express, so they are refused
  {
    int with_neumann = 0;
    for (int i = 0; i < n; ++i) {
      bool nm = false;
      for (int64_t f = face_ptr[i]; f < face_ptr[i + 1] && !nm; ++f) nm = m->fbc[f] == HHO_FACE_NEUMANN;
      with_neumann += nm;
    }
    if (with_neumann != 0 && with_neumann != n)
      hho::fail(HHO_E_INVALID_ARG, "set_segments: either every member or none may have Neumann faces");
  }
  // the default penalty 4(k+1)(k+d)/d max card(F_T) is taken per member
  p->cell_eta.clear();
  if (!(p->opt.eta > 0)) {
    const int d = p->d, k = p->k;
    p->cell_eta.resize(m->nc);
    for (int i = 0; i < n; ++i) {
      int64_t mf = 0;
      for (int64_t c = cell_ptr[i]; c < cell_ptr[i + 1]; ++c) mf = std::max<int64_t>(mf, m->cptr[c + 1] - m->cptr[c]);
      const double eta_i = 4.0 * (k + 1) * (k + d) / d * (double)mf;
      for (int64_t c = cell_ptr[i]; c < cell_ptr[i + 1]; ++c) p->cell_eta[c] = eta_i;
    }
  }
  p->nseg = n;
  p->seg_face_ptr.assign(face_ptr, face_ptr + n + 1);
  p->seg_cell_ptr.assign(cell_ptr, cell_ptr + n + 1);
  hho::init_levels(p);  // the coarse solver choice depends on the segments
  p->segl.assign(p->nlev, hho::SegLevel{});
  for (int l = 0; l < p->nlev; ++l) {
    const hho::LevelInfo &L = p->lev[l];
    const int64_t dp = (int64_t)p->d * L.p;
    hho::SegLevel &S = p->segl[l];
    S.hseg.resize(n);
    S.hptr.assign(1, 0);
    for (int i = 0; i < n; ++i) {
      hho::SegInfo &g = S.hseg[i];
      g.fo = face_ptr[i] * dp;
      g.fl = (face_ptr[i + 1] - face_ptr[i]) * dp;
      g.co = L.nface + cell_ptr[i] * L.t;
      g.cl = (cell_ptr[i + 1] - cell_ptr[i]) * L.t;
      const int64_t len = g.fl + g.cl;
      if (len > INT32_MAX) hho::fail(HHO_E_INVALID_ARG, "set_segments: segment too large");
      for (int64_t e = 0; e < len; e += hho::kSegChunk)
        S.hch.push_back({i, (int32_t)e, (int32_t)std::min<int64_t>(hho::kSegChunk, len - e), 0});
      S.hptr.push_back((int32_t)S.hch.size());
    }
  }
  p->hseg = p->segl[0].hseg;
  p->hchunks = p->segl[0].hch;
  p->hchunk_ptr = p->segl[0].hptr;
  return HHO_OK;
  ABI_END
}

int hho_batch_results(const hho_problem *p, int *iters, double *rel, int n) {
  ABI_BEGIN
  if (!p || n != p->nseg || p->seg_its.empty()) hho::fail(HHO_E_INVALID_ARG, "batch_results: no batched solve");
  for (int i = 0; i < n; ++i) {
    if (iters) iters[i] = p->seg_its[i];
    if (rel) rel[i] = p->seg_rel[i];
  }
  return HHO_OK;
  ABI_END
}

// ------------------------------------------------------------ batches built from separate problems
struct hho_batch {
  std::unique_ptr<hho_mesh> mesh;  // disjoint union of the members' meshes
  hho_problem *P = nullptr;        // the combined problem (owned)
  int n = 0;
  std::vector<int64_t> foff, coff;  // first face / cell of every member in the union, n+1 entries
  ~hho_batch() { hho_problem_destroy(P); }
};

static bool same_solver_options(const hho_options &a, const hho_options &b) {
  return a.rtol == b.rtol && a.max_it == b.max_it && a.restart == b.restart && a.smooth_its == b.smooth_its &&
         a.precision == b.precision && a.coarse_mode == b.coarse_mode && a.coarse_rtol == b.coarse_rtol &&
         a.coarse_restart == b.coarse_restart && a.coarse_max_it == b.coarse_max_it && a.quad_extra == b.quad_extra &&
         a.coarse_amg_sweeps == b.coarse_amg_sweeps && a.learned == b.learned &&
         a.coarse_amg_explicit == b.coarse_amg_explicit && a.coarse_amg_psmooth == b.coarse_amg_psmooth &&
         a.smoother == b.smoother && a.nullspace == b.nullspace && a.vcycle_copy == b.vcycle_copy &&
         a.local_build == b.local_build;
}

int hho_batch_create(hho_problem *const *ps, int n, hho_batch **out) {
  ABI_BEGIN
  if (!ps || n < 1 || !out) hho::fail(HHO_E_INVALID_ARG, "batch_create: bad argument");
  *out = nullptr;
  const hho_problem *p0 = ps[0];
  for (int i = 0; i < n; ++i) {
    const hho_problem *q = ps[i];
    if (!q) hho::fail(HHO_E_INVALID_ARG, "batch_create: NULL member");
    if (!q->have_data) hho::fail(HHO_E_INVALID_ARG, "batch_create: every member needs hho_problem_set_data first");
    if (q->nseg > 0) hho::fail(HHO_E_INVALID_ARG, "batch_create: a member is itself a batch");
    if (q->d != p0->d || q->k != p0->k || q->cond != p0->cond || q->deg != p0->deg)
      hho::fail(HHO_E_INVALID_ARG, "batch_create: members differ in dimension, degree schedule or condensation");
    if (!same_solver_options(q->opt, p0->opt))
      hho::fail(HHO_E_INVALID_ARG, "batch_create: members differ in solver options (only eta may differ)");
  }
  auto B = std::make_unique<hho_batch>();
  B->n = n;
  B->foff.resize(n + 1);
  B->coff.resize(n + 1);
  std::vector<hho_mesh_desc> descs(n);
  for (int i = 0; i < n; ++i) {
    const hho_mesh *m = ps[i]->mesh;
    descs[i] = hho_mesh_desc{m->dim, m->nv, m->verts.data(), m->nf, m->fptr.data(), m->fvtx.data(),
                             m->nc, m->cptr.data(), m->cface.data(), m->fbc.data()};
  }
  B->mesh = std::make_unique<hho_mesh>();
  build_union_mesh(descs.data(), n, B->mesh.get(), B->foff.data(), B->coff.data());
  hho_options opt = p0->opt;
  opt.eta = 1.0;  // the members' local operators are copied below, each with its own penalty
  hho_problem *P = nullptr;
  int rc = hho_problem_create(B->mesh.get(), p0->k, p0->cond, p0->nlev, p0->deg.data(), &opt, &P);
  if (rc != HHO_OK) return rc;
  B->P = P;
  rc = hho_problem_set_segments(P, n, B->foff.data(), B->coff.data());
  if (rc != HHO_OK) return rc;
  // local operators: the members' records (or, for the device build, their data
  // moments and penalties), concatenated in union cell order
  for (int i = 0; i < n; ++i)
    if (ps[i]->local_dev != p0->local_dev)
      hho::fail(HHO_E_INVALID_ARG, "batch_create: members differ in where their local operators are built");
  P->local_dev = p0->local_dev;
  if (P->local_dev) {
    const int64_t nfu = B->mesh->nf;
    hho::DataMoments &D = P->dmom;
    D = hho::DataMoments{};
    D.foff.assign(nfu, -1);
    P->cell_eta_dev.clear();
    for (int i = 0; i < n; ++i) {
      const hho_problem *q = ps[i];
      const int64_t base = (int64_t)D.fd.size();
      D.mf.insert(D.mf.end(), q->dmom.mf.begin(), q->dmom.mf.end());
      D.fd.insert(D.fd.end(), q->dmom.fd.begin(), q->dmom.fd.end());
      for (int64_t f = 0; f < q->mesh->nf; ++f)
        if (q->dmom.foff[f] >= 0) D.foff[B->foff[i] + f] = base + q->dmom.foff[f];
      P->cell_eta_dev.insert(P->cell_eta_dev.end(), q->cell_eta_dev.begin(), q->cell_eta_dev.end());
      if (!q->user_rhs.empty()) hho::fail(HHO_E_INVALID_ARG, "batch_create: a member has hho_set_moments data");
    }
    const int qdeg = 2 * p0->k + 2 + std::max(0, p0->opt.quad_extra);
    if (!hho::choose_local_device(P, qdeg))
      hho::fail(HHO_E_INVALID_ARG, "batch_create: the union cannot use the device build of its members");
  }
  hho::LocalData &L = P->loc;
  L = hho::LocalData{};
  const hho::LocalData &L0 = p0->loc;
  L.k = L0.k;
  L.d = L0.d;
  L.nT = L0.nT;
  L.nF = L0.nF;
  L.N1 = L0.N1;
  L.off.assign(1, 0);
  for (int i = 0; i < n; ++i) {
    const hho::LocalData &Li = ps[i]->loc;
    const int64_t base = L.off.back();
    L.rec.insert(L.rec.end(), Li.rec.begin(), Li.rec.end());
    L.nloc.insert(L.nloc.end(), Li.nloc.begin(), Li.nloc.end());
    for (size_t c = 1; c < Li.off.size(); ++c) L.off.push_back(base + Li.off[c]);
  }
  P->opt.eta = p0->opt.eta;
  P->cell_eta.clear();
  hho::settle_auto_coarse(P);
  hho::amg_levels(P);
  P->have_data = true;
  P->setup_done = false;
  hho::Arena A;
  hho::plan(P, A);
  P->need = A.off + 256;
  *out = B.release();
  return HHO_OK;
  ABI_END
}

void hho_batch_destroy(hho_batch *b) { delete b; }

int hho_batch_problem(hho_batch *b, hho_problem **p) {
  ABI_BEGIN
  if (!b || !p) hho::fail(HHO_E_INVALID_ARG, "batch_problem: NULL");
  *p = b->P;
  return HHO_OK;
  ABI_END
}

int hho_batch_sizes(const hho_batch *b, int64_t *face_n, int64_t *p_n) {
  ABI_BEGIN
  if (!b || !face_n || !p_n) hho::fail(HHO_E_INVALID_ARG, "batch_sizes: NULL");
  const hho::LevelInfo &L0 = b->P->lev[0];
  const int64_t fdof = L0.nface / b->mesh->nf;  // d * n_F per face
  for (int i = 0; i < b->n; ++i) {
    face_n[i] = (b->foff[i + 1] - b->foff[i]) * fdof;
    p_n[i] = (b->coff[i + 1] - b->coff[i]) * L0.t;
  }
  return HHO_OK;
  ABI_END
}

int hho_batch_solve(hho_batch *b, double *face_out, const int64_t *face_off, double *p_out, const int64_t *p_off,
                    int *iters, double *hist, const int64_t *hist_off, double *final_rel, int *status) {
  ABI_BEGIN
  if (!b || !face_out || !face_off || !p_out || !p_off) hho::fail(HHO_E_INVALID_ARG, "batch_solve: NULL argument");
  hho_problem *P = b->P;
  need_setup(P);
  const int n = b->n;
  const hho::LevelInfo &L0 = P->lev[0];
  const int64_t fdof = L0.nface / b->mesh->nf;
  for (int i = 0; i < n; ++i) {
    const int64_t fn = (b->foff[i + 1] - b->foff[i]) * fdof, pn = (b->coff[i + 1] - b->coff[i]) * L0.t;
    if (face_off[i + 1] - face_off[i] < fn || p_off[i + 1] - p_off[i] < pn) {
      hho::set_error("batch_solve: output range of member " + std::to_string(i) + " too small: " +
                     std::to_string(fn) + " face and " + std::to_string(pn) + " pressure values are needed");
      return HHO_E_CAPACITY;
    }
    if (hist_off && hist_off[i + 1] < hist_off[i]) hho::fail(HHO_E_INVALID_ARG, "batch_solve: decreasing hist_off");
  }
  P->opt_seg_hist = hist && hist_off;
  int its = 0;
  double rel = 0;
  const int rc = hho::fgmres_batched(P, nullptr, &its, nullptr, 0, &rel);
  P->opt_seg_hist = false;
  for (int i = 0; i < n; ++i) {
    const int64_t fn = (b->foff[i + 1] - b->foff[i]) * fdof, pn = (b->coff[i + 1] - b->coff[i]) * L0.t;
    HIPCHK(hipMemcpyAsync(face_out + face_off[i], P->ox + b->foff[i] * fdof, fn * sizeof(double),
                          hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipMemcpyAsync(p_out + p_off[i], P->ox + L0.nface + b->coff[i] * L0.t, pn * sizeof(double),
                          hipMemcpyDeviceToHost, P->stream));
  }
  HIPCHK(hipStreamSynchronize(P->stream));
  for (int i = 0; i < n; ++i) {
    if (iters) iters[i] = P->seg_its[i];
    if (final_rel) final_rel[i] = P->seg_rel[i];
    if (status) status[i] = P->seg_rel[i] <= P->opt.rtol ? HHO_OK : HHO_E_NOT_CONVERGED;
    if (hist && hist_off) {
      const std::vector<double> &h = P->seg_hist_h[i];
      const int64_t cap = hist_off[i + 1] - hist_off[i];
      for (int64_t e = 0; e < cap && e < (int64_t)h.size(); ++e) hist[hist_off[i] + e] = h[e];
    }
  }
  return rc;
  ABI_END
}

// ------------------------------------------------------------ learned parameters as bytes
namespace {
constexpr char kMlpMagic[8] = {'H', 'H', 'O', 'M', 'L', 'P', '0', '1'};
struct MlpFileHeader {
  char magic[8];
  int32_t n_in, n_out, hidden, reserved;
  int64_t n_params;
};
}  // namespace

int hho_learned_save(const hho_problem *p, void *buf, size_t cap, size_t *need) {
  ABI_BEGIN
  need_learned(p);
  if (!p->learned_ready) hho::fail(HHO_E_INVALID_ARG, "learned_save: no parameters set");
  const int64_t np = hho::mlp_param_count(p->md);
  const size_t bytes = sizeof(MlpFileHeader) + (size_t)np * sizeof(float);
  if (need) *need = bytes;
  if (!buf || cap < bytes) {
    hho::set_error("learned_save: the buffer needs " + std::to_string(bytes) + " bytes");
    return HHO_E_CAPACITY;
  }
  MlpFileHeader h{};
  std::memcpy(h.magic, kMlpMagic, 8);
  h.n_in = p->md.n_in;
  h.n_out = p->md.n_out;
  h.hidden = hho::kMlpHidden;
  h.n_params = np;
  std::memcpy(buf, &h, sizeof(h));
  HIPCHK(hipMemcpyAsync((char *)buf + sizeof(h), p->mlp_prm, np * sizeof(float), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return HHO_OK;
  ABI_END
}

int hho_learned_load(hho_problem *p, const void *buf, size_t n) {
  ABI_BEGIN
  need_learned(p);
  if (!buf || n < sizeof(MlpFileHeader)) hho::fail(HHO_E_INVALID_ARG, "learned_load: buffer too short");
  MlpFileHeader h;
  std::memcpy(&h, buf, sizeof(h));
  const int64_t np = hho::mlp_param_count(p->md);
  if (std::memcmp(h.magic, kMlpMagic, 8) != 0) hho::fail(HHO_E_INVALID_ARG, "learned_load: not a saved network");
  if (h.n_in != p->md.n_in || h.n_out != p->md.n_out || h.hidden != hho::kMlpHidden || h.n_params != np)
    hho::fail(HHO_E_INVALID_ARG, "learned_load: the network's sizes differ from this problem's");
  if (n < sizeof(h) + (size_t)np * sizeof(float)) hho::fail(HHO_E_INVALID_ARG, "learned_load: buffer too short");
  return hho_learned_set_params(p, (const float *)((const char *)buf + sizeof(h)), np);
  ABI_END
}

// ------------------------------------------------------------ right-hand sides given as moments
int hho_moments_size(const hho_problem *p, int64_t *n_u, int64_t *n_p) {
  ABI_BEGIN
  if (!p || !n_u || !n_p) hho::fail(HHO_E_INVALID_ARG, "moments_size: NULL");
  if (!p->have_data) hho::fail(HHO_E_INVALID_ARG, "moments_size: call hho_problem_set_data first");
  int64_t nu = 0;
  for (int32_t v : p->loc.nloc) nu += (int64_t)p->d * v;
  *n_u = nu;
  *n_p = (int64_t)p->mesh->nc * p->loc.nT;
  return HHO_OK;
  ABI_END
}

int hho_set_moments(hho_problem *p, const double *rhs_u, const double *rhs_p) {
  ABI_BEGIN
  if (!p || !rhs_u || !rhs_p) hho::fail(HHO_E_INVALID_ARG, "set_moments: NULL");
  if (!p->have_data) hho::fail(HHO_E_INVALID_ARG, "set_moments: call hho_problem_set_data first");
  hho::LocalData &L = p->loc;
  const int d = p->d, nT = L.nT;
  int64_t ou = 0;
  if (p->local_dev) {  // kept on the host, written over the device-built records at hho_setup
    const int64_t nc = p->mesh->nc;
    p->user_off.assign(nc + 1, 0);
    for (int64_t c = 0; c < nc; ++c) p->user_off[c + 1] = p->user_off[c] + (int64_t)d * L.nloc[c] + nT;
    p->user_rhs.resize(p->user_off[nc]);
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t nl = L.nloc[c];
      std::memcpy(&p->user_rhs[p->user_off[c]], rhs_u + ou, sizeof(double) * d * nl);
      std::memcpy(&p->user_rhs[p->user_off[c] + d * nl], rhs_p + c * nT, sizeof(double) * nT);
      ou += d * nl;
    }
    p->uploaded = false;
    p->setup_done = false;
    return HHO_OK;
  }
  for (int64_t c = 0; c < p->mesh->nc; ++c) {
    const int64_t nl = L.nloc[c];
    double *r = L.rec.data() + L.off[c] + nl * nl + (int64_t)d * nT * nl;  // [rhs_u (d*nloc) | rhs_p (nT)]
    std::memcpy(r, rhs_u + ou, sizeof(double) * d * nl);
    std::memcpy(r + d * nl, rhs_p + c * nT, sizeof(double) * nT);
    ou += d * nl;
  }
  p->uploaded = false;  // the next hho_setup copies the records again
  p->setup_done = false;
  return HHO_OK;
  ABI_END
}

