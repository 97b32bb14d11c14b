// Device side of the coarsest level's sparse direct solver (pointers into the
// workspace; the index arrays come from the symbolic phase, direct.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "direct.h"
#include "probe.h"

namespace hho {

struct NdDev {
  const int32_t *m = nullptr, *nfs = nullptr, *child = nullptr;
  const int64_t *off = nullptr, *voff = nullptr, *dofoff = nullptr, *soff = nullptr;
  const int32_t *dof = nullptr, *cmap = nullptr;
  const int64_t *src = nullptr, *dst = nullptr;
  const int32_t *hfront = nullptr, *tiles = nullptr, *chunks = nullptr, *schunks = nullptr;
  double *F = nullptr;  // fronts, m*m each, row-major
  double *V = nullptr;  // solve vectors, m each
  double *S = nullptr;  // panel scratch of the height being eliminated
  double *coef = nullptr;  // per member: projection coefficient of the right-hand side on its null vector
  const int64_t *pins = nullptr, *segp = nullptr;  // per member: pinned unknown; cell ranges
  const int32_t *cseg = nullptr;                   // member of every cell
  int64_t npair = 0;
};

// Numeric factorisation: fronts cleared, operator entries placed, then each
// height eliminated (children before parents).  err: first front with a zero or
// non-finite pivot, plus one.
void launch_nd_factor(const NdHost &H, const NdDev &D, const DLevel<double> &L, int64_t nb, int64_t ncpl,
                      int *err, hipStream_t s);
// x = S^{-1} b on the coarsest level; with pinned unknowns (each member's
// constant-pressure null space, zmean the null vectors' cell coefficients) b is
// first made orthogonal to every member's null vector and so is x afterwards.
// probe: live timing of the passes (classes HHO_PROBE_DIRECT_FWD / _BWD, level = tree height), or null.
void launch_nd_solve(const NdHost &H, const NdDev &D, int64_t nface, int t, const double *zmean, const double *b,
                     double *x, hipStream_t s, KernelProbe *probe);

}  // namespace hho
