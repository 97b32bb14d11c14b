// Smoothed-aggregation hierarchy for the velocity block of the coarsest level.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace hho {

constexpr double kAmgOmegaSA = 4.0 / 3.0;   // prolongator smoothing weight (divided by lambda)
constexpr double kAmgOmegaJac = 4.0 / 3.0;  // damped-Jacobi smoother weight (divided by lambda)
constexpr int kAmgCoarsest = 128;           // dense inverse at or below this size
constexpr int kAmgMaxRowNnz = 160;          // stop coarsening before a level this dense (entries per row)
constexpr int kAmgCoarseSweeps = 6;         // Jacobi sweeps on a coarsest level above kAmgCoarsest
constexpr int kAmgPowerSteps = 15;          // power iterations for lambda ~ rho(D^{-1} A)
constexpr double kAmgLambdaSafety = 1.05;

struct AmgHostLevel {
  int n = 0, nc = 0;                     // rows; aggregates (0 on the coarsest level)
  std::vector<int32_t> rp, ci, diag;     // A pattern, diagonal positions
  std::vector<int32_t> agg;              // aggregate of every row
  std::vector<int32_t> prp, pci;         // P pattern (n x nc)
  std::vector<int32_t> pgp, pgi;         // A entries summed into each P entry
  std::vector<int32_t> pself;            // 1 where the entry is the tentative injection
  int np1 = 0;                           // two smoothing steps: entries of P_1 (the gathers
                                         // above, pself, p1row refer to P_1), else 0
  std::vector<int32_t> p1row;            // row of every P_1 entry
  std::vector<int32_t> qpp, qpa, qpb;    // B_1 = A P_1 in the final P pattern: pairs (A entry, P_1 entry)
  std::vector<int32_t> p2src;            // final P entry -> its P_1 entry, or -1
  std::vector<int32_t> ptp, pti, pte;    // P^T by coarse row: fine row, P entry
  std::vector<int32_t> brp, bci;         // B = A P pattern
  std::vector<int32_t> bpp, bpa, bpb;    // B pairs (A entry, P entry)
  std::vector<int32_t> btp, bti, bte;    // B^T by coarse row: fine row, B entry
  std::vector<int32_t> cpp, cpa, cpb;    // next A pairs (P entry, B entry)
};

struct AmgHost {
  std::vector<AmgHostLevel> levels;
};

void amg_symbolic(int n0, const int32_t *rp0, const int32_t *ci0, int coarsest, int p_steps, AmgHost *H);

}  // namespace hho
