// Symbolic phase of the smoothed-aggregation hierarchy used by the coarsest
// level's block preconditioner.  Everything here depends on the sparsity
// pattern only (mesh topology), so it is built once per problem; the device
// computes every value (see k_amg.hip).
//
// Level l holds A_l (CSR, sorted columns), the aggregates of its rows (an
// unaggregated row in index order opens an aggregate holding itself and its
// unaggregated neighbours in the aggregation graph G_l, with G_0 the pattern of
// A_0 and G_{l+1} the pattern of T^T G_l T), the pattern of P = T - w D^{-1} A T (T the 0/1
// aggregate injection), and the gather lists that evaluate
//   P        (entries of A summed per (row, aggregate)),
//   B = A P  (pairs (A entry, P entry)),
//   A_{l+1} = P^T B  (pairs (P entry, B entry)).
#include <algorithm>
#include <map>

#include "amg.h"

namespace hho {

static void csr_from_rows(const std::vector<std::vector<int32_t>> &rows, std::vector<int32_t> &rp,
                          std::vector<int32_t> &ci) {
  rp.assign(rows.size() + 1, 0);
  for (size_t i = 0; i < rows.size(); ++i) rp[i + 1] = rp[i] + (int32_t)rows[i].size();
  ci.resize(rp.back());
  for (size_t i = 0; i < rows.size(); ++i) std::copy(rows[i].begin(), rows[i].end(), ci.begin() + rp[i]);
}

void amg_symbolic(int n0, const int32_t *rp0, const int32_t *ci0, int coarsest, AmgHost *H) {
  H->levels.clear();
  std::vector<int32_t> rp(rp0, rp0 + n0 + 1), ci(ci0, ci0 + rp0[n0]);
  std::vector<int32_t> grp = rp, gci = ci;  // aggregation graph (pattern of T^T G T)
  int n = n0;
  for (;;) {
    AmgHostLevel L;
    L.n = n;
    L.rp = rp;
    L.ci = ci;
    L.diag.assign(n, -1);
    for (int i = 0; i < n; ++i)
      for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] == i) L.diag[i] = e;
    for (int i = 0; i < n; ++i)
      if (L.diag[i] < 0) fail(HHO_E_MESH, "coarse operator pattern lacks a diagonal entry");
    if (n <= coarsest) {
      L.nc = 0;
      H->levels.push_back(std::move(L));
      break;
    }
    // aggregation
    L.agg.assign(n, -1);
    int na = 0;
    for (int i = 0; i < n; ++i) {
      if (L.agg[i] >= 0) continue;
      for (int e = grp[i]; e < grp[i + 1]; ++e)
        if (L.agg[gci[e]] < 0) L.agg[gci[e]] = na;
      L.agg[i] = na;
      ++na;
    }
    if (na >= n) {  // no coarsening possible: make this the coarsest level
      L.nc = 0;
      L.agg.clear();
      H->levels.push_back(std::move(L));
      break;
    }
    L.nc = na;
    // P pattern and its gather lists (A entries per (row, aggregate))
    std::vector<std::vector<int32_t>> prow(n);
    std::vector<std::vector<std::vector<int32_t>>> plist(n);
    for (int i = 0; i < n; ++i) {
      std::map<int32_t, std::vector<int32_t>> m;
      m[L.agg[i]];  // T contributes (i, agg[i]) even if nothing else does
      for (int e = rp[i]; e < rp[i + 1]; ++e) m[L.agg[ci[e]]].push_back(e);
      for (auto &kv : m) {
        prow[i].push_back(kv.first);
        plist[i].push_back(kv.second);
      }
    }
    csr_from_rows(prow, L.prp, L.pci);
    L.pgp.assign(L.pci.size() + 1, 0);
    for (int i = 0, k = 0; i < n; ++i)
      for (auto &lst : plist[i]) {
        L.pgp[k + 1] = L.pgp[k] + (int32_t)lst.size();
        L.pgi.insert(L.pgi.end(), lst.begin(), lst.end());
        ++k;
      }
    L.pself.resize(L.pci.size());
    for (int i = 0; i < n; ++i)
      for (int e = L.prp[i]; e < L.prp[i + 1]; ++e) L.pself[e] = (L.pci[e] == L.agg[i]) ? 1 : 0;
    // P^T (by coarse column): rows i and P entry indices
    std::vector<std::vector<std::pair<int32_t, int32_t>>> pt(na);
    for (int i = 0; i < n; ++i)
      for (int e = L.prp[i]; e < L.prp[i + 1]; ++e) pt[L.pci[e]].push_back({i, e});
    L.ptp.assign(na + 1, 0);
    for (int I = 0; I < na; ++I) {
      L.ptp[I + 1] = L.ptp[I] + (int32_t)pt[I].size();
      for (auto &pr : pt[I]) {
        L.pti.push_back(pr.first);
        L.pte.push_back(pr.second);
      }
    }
    // B = A P : pattern + pairs (A entry, P entry)
    std::vector<std::vector<int32_t>> brow(n);
    std::vector<std::vector<std::vector<std::pair<int32_t, int32_t>>>> bpairs(n);
    for (int i = 0; i < n; ++i) {
      std::map<int32_t, std::vector<std::pair<int32_t, int32_t>>> m;
      for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        for (int pe = L.prp[j]; pe < L.prp[j + 1]; ++pe) m[L.pci[pe]].push_back({e, pe});
      }
      for (auto &kv : m) {
        brow[i].push_back(kv.first);
        bpairs[i].push_back(kv.second);
      }
    }
    csr_from_rows(brow, L.brp, L.bci);
    L.bpp.assign(L.bci.size() + 1, 0);
    for (int i = 0, k = 0; i < n; ++i)
      for (auto &lst : bpairs[i]) {
        L.bpp[k + 1] = L.bpp[k] + (int32_t)lst.size();
        for (auto &pr : lst) {
          L.bpa.push_back(pr.first);
          L.bpb.push_back(pr.second);
        }
        ++k;
      }
    // A_next = P^T B : pattern + pairs (P entry, B entry)
    std::vector<std::vector<int32_t>> crow(na);
    std::vector<std::vector<std::vector<std::pair<int32_t, int32_t>>>> cpairs(na);
    for (int I = 0; I < na; ++I) {
      std::map<int32_t, std::vector<std::pair<int32_t, int32_t>>> m;
      for (int k = L.ptp[I]; k < L.ptp[I + 1]; ++k) {
        const int i = L.pti[k], pe = L.pte[k];
        for (int be = L.brp[i]; be < L.brp[i + 1]; ++be) m[L.bci[be]].push_back({pe, be});
      }
      for (auto &kv : m) {
        crow[I].push_back(kv.first);
        cpairs[I].push_back(kv.second);
      }
    }
    std::vector<int32_t> nrp, nci;
    csr_from_rows(crow, nrp, nci);
    L.cpp.assign(nci.size() + 1, 0);
    for (int I = 0, k = 0; I < na; ++I)
      for (auto &lst : cpairs[I]) {
        L.cpp[k + 1] = L.cpp[k] + (int32_t)lst.size();
        for (auto &pr : lst) {
          L.cpa.push_back(pr.first);
          L.cpb.push_back(pr.second);
        }
        ++k;
      }
    // next aggregation graph: aggregates adjacent when any of their members are
    std::vector<std::vector<int32_t>> grow(na);
    for (int i = 0; i < n; ++i)
      for (int e = grp[i]; e < grp[i + 1]; ++e) grow[L.agg[i]].push_back(L.agg[gci[e]]);
    for (auto &r : grow) {
      std::sort(r.begin(), r.end());
      r.erase(std::unique(r.begin(), r.end()), r.end());
    }
    csr_from_rows(grow, grp, gci);
    H->levels.push_back(std::move(L));
    rp = nrp;
    ci = nci;
    n = na;
  }
}

}  // namespace hho
