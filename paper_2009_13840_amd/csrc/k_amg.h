// Device-side smoothed-aggregation hierarchy (pointers into the workspace).
#pragma once

#include "probe.h"

#include <hip/hip_runtime.h>

#include <cstdint>

#include "amg.h"
#include "device.h"

namespace hho {

constexpr int kMaxAmgLevels = 16;

struct AmgDevLevel {
  int n = 0, nc = 0;
  int64_t nnz = 0, npe = 0, nbe = 0;
  const int32_t *rp = nullptr, *ci = nullptr, *diag = nullptr;
  double *val = nullptr, *dinv = nullptr, *lam = nullptr;
  const int32_t *prp = nullptr, *pci = nullptr, *prow = nullptr, *pgp = nullptr, *pgi = nullptr, *pself = nullptr;
  double *pval = nullptr;
  // two prolongator smoothing steps (np1 > 0): P_1 (np1 entries, gathered by
  // pgp/pgi/pself, rows p1row), B_1 = A P_1 on the final P pattern (pairs
  // qpp/qpa/qpb), P = P_1 (via p2src) - w D^{-1} B_1
  int np1 = 0;
  const int32_t *p1row = nullptr, *qpp = nullptr, *qpa = nullptr, *qpb = nullptr, *p2src = nullptr;
  double *pval1 = nullptr, *qval = nullptr;
  const int32_t *ptp = nullptr, *pti = nullptr, *pte = nullptr;
  const int32_t *bpp = nullptr, *bpa = nullptr, *bpb = nullptr;
  const int32_t *brp = nullptr, *bci = nullptr;              // B = A P by rows
  const int32_t *btp = nullptr, *bti = nullptr, *bte = nullptr;  // B^T by coarse rows
  double *bval = nullptr;
  double *ptval = nullptr, *btval = nullptr;  // P and B values in P^T / B^T order
  const int32_t *cpp = nullptr, *cpa = nullptr, *cpb = nullptr;
  double *x = nullptr, *r = nullptr, *res = nullptr, *tmp = nullptr;  // [n][d]
};

constexpr int kAmgExplicitMax = 4096;  // largest level replaced by its explicit V-cycle matrix

struct AmgDev {
  int nlev = 0;
  AmgDevLevel lev[kMaxAmgLevels];
  // explicit operator M of the V-cycle on level expl (-1: none), [n][n] row-major
  // (it is cx[expl]), and the column blocks [n_l][n_expl] it is formed with
  int expl = -1;
  double *mexpl = nullptr;
  double *cr[kMaxAmgLevels] = {}, *cx[kMaxAmgLevels] = {}, *ct[kMaxAmgLevels] = {};
  double *ainv = nullptr, *dense_scratch = nullptr, *partial = nullptr;  // partial: 2 x 256 power-step sums
  KernelProbe *probe = nullptr;  // live timing of armed kernel classes (may be null)
};

void amg_numeric_setup(const AmgDev &A, int cond, int d, int bs, int64_t nnzb0, const double *bsr0, int nu,
                       int *err, hipStream_t s);
void bp_setup(const DTopo &tp, int cond, const int32_t *fdiag, const double *bsr, const double *cpl, double *Sd,
              hipStream_t s);
// z = block preconditioner applied to v (coarsest-level vectors in the global layout).
// skip (device, may be null): when *skip is nonzero at launch time every kernel of
// the application returns at once (a Krylov process that has already converged
// inside a chunk of queued iterations).
void bp_apply(const DTopo &tp, const AmgDev &A, int64_t nface, const double *cpl, const double *Sd, const double *v,
              double *z, int nu, hipStream_t s, const int *skip = nullptr);

}  // namespace hho
