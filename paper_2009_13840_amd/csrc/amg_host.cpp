// Symbolic phase of the smoothed-aggregation hierarchy used by the coarsest
// level's block preconditioner.  Everything here depends on the sparsity
// pattern only (mesh topology), so it is built once per problem; the device
// computes every value (see k_amg.hip).
//
// Level l holds A_l (CSR, sorted columns), the aggregates of its rows (an
// unaggregated row in index order opens an aggregate holding itself and its
// unaggregated neighbours in the aggregation graph G_l, with G_0 the pattern of
// A_0 and G_{l+1} the pattern of T^T G_l T), the pattern of P = T - w D^{-1} A T (T the 0/1
// aggregate injection; with two smoothing steps P = P_1 - w D^{-1} A P_1 from that
// P_1), and the gather lists that evaluate
//   P        (entries of A summed per (row, aggregate); second step: pairs of A P_1),
//   B = A P  (pairs (A entry, P entry)),
//   A_{l+1} = P^T B  (pairs (P entry, B entry)).
#include <algorithm>

#include "amg.h"

namespace hho {

// Entries (column, first source, second source) of one output row, grouped by
// column: columns ascending and, within a column, the entries in the order they
// were produced (the device sums them in that order).  Grouping counts the
// entries per distinct column (a column -> slot map kept across rows) and sorts
// only the distinct columns.
struct RowGroups {
  struct E {
    int32_t col, a, b;
  };
  std::vector<E> e;
  std::vector<int32_t> slot;  // column -> index in ucol, -1 when absent (grown on demand)
  std::vector<int32_t> ucol, cnt, pos, order;
  void add(int32_t col, int32_t a, int32_t b) { e.push_back({col, a, b}); }
  // appends the row to (cols, pair offsets, pair lists)
  // (skip_negative: entries whose first source is < 0 only create their column)
  void flush(std::vector<int32_t> &cols, std::vector<int32_t> &pp, std::vector<int32_t> &pa,
             std::vector<int32_t> *pb, bool skip_negative = false) {
    for (const E &x : e) {
      if (x.col >= (int32_t)slot.size()) slot.resize((size_t)x.col + 1, -1);
      int32_t &sl = slot[x.col];
      if (sl < 0) {
        sl = (int32_t)ucol.size();
        ucol.push_back(x.col);
        cnt.push_back(0);
      }
      if (!(skip_negative && x.a < 0)) ++cnt[sl];
    }
    order.resize(ucol.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::sort(order.begin(), order.end(), [&](int32_t u, int32_t v) { return ucol[u] < ucol[v]; });
    pos.resize(ucol.size());
    int32_t base = (int32_t)pa.size();
    for (int32_t o : order) {
      cols.push_back(ucol[o]);
      pp.push_back(base);
      pos[o] = base;
      base += cnt[o];
    }
    pa.resize(base);
    if (pb) pb->resize(base);
    for (const E &x : e) {
      if (skip_negative && x.a < 0) continue;
      const int32_t q = pos[slot[x.col]]++;
      pa[q] = x.a;
      if (pb) (*pb)[q] = x.b;
    }
    for (int32_t c : ucol) slot[c] = -1;
    ucol.clear();
    cnt.clear();
    e.clear();
  }
};

void amg_symbolic(int n0, const int32_t *rp0, const int32_t *ci0, int coarsest, int p_steps, AmgHost *H) {
  H->levels.clear();
  std::vector<int32_t> rp(rp0, rp0 + n0 + 1), ci(ci0, ci0 + rp0[n0]);
  std::vector<int32_t> grp = rp, gci = ci;  // aggregation graph (pattern of T^T G T)
  int n = n0;
  RowGroups rg;
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
    // P pattern and its gather lists (A entries summed per (row, aggregate));
    // the tentative entry (i, agg[i]) exists even if no A entry falls in it
    L.prp.assign(1, 0);
    for (int i = 0; i < n; ++i) {
      rg.add(L.agg[i], -1, 0);
      for (int e = rp[i]; e < rp[i + 1]; ++e) rg.add(L.agg[ci[e]], e, 0);
      rg.flush(L.pci, L.pgp, L.pgi, nullptr, /*skip_negative=*/true);
      L.prp.push_back((int32_t)L.pci.size());
    }
    L.pgp.push_back((int32_t)L.pgi.size());
    L.pself.resize(L.pci.size());
    for (int i = 0; i < n; ++i)
      for (int e = L.prp[i]; e < L.prp[i + 1]; ++e) L.pself[e] = (L.pci[e] == L.agg[i]) ? 1 : 0;
    // second smoothing step: with P_1 as above and B_1 = A P_1 (pairs (A entry,
    // P_1 entry)), P = P_1 - w D^{-1} B_1 on the pattern of B_1, which holds that
    // of P_1 (A has its diagonal); p2src gives each entry's P_1 entry or -1
    auto second_step = [&]() {
      L.np1 = (int)L.pci.size();
      L.p1row.resize(L.np1);
      for (int i = 0; i < n; ++i)
        for (int e = L.prp[i]; e < L.prp[i + 1]; ++e) L.p1row[e] = i;
      std::vector<int32_t> qrp(1, 0), qci;
      L.qpp.clear();
      L.qpa.clear();
      L.qpb.clear();
      for (int i = 0; i < n; ++i) {
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
          const int j = ci[e];
          for (int pe = L.prp[j]; pe < L.prp[j + 1]; ++pe) rg.add(L.pci[pe], e, pe);
        }
        rg.flush(qci, L.qpp, L.qpa, &L.qpb);
        qrp.push_back((int32_t)qci.size());
      }
      L.qpp.push_back((int32_t)L.qpa.size());
      L.p2src.assign(qci.size(), -1);
      for (int i = 0; i < n; ++i) {  // both rows sorted by column
        int e1 = L.prp[i];
        for (int e = qrp[i]; e < qrp[i + 1]; ++e) {
          while (e1 < L.prp[i + 1] && L.pci[e1] < qci[e]) ++e1;
          if (e1 < L.prp[i + 1] && L.pci[e1] == qci[e]) L.p2src[e] = e1;
        }
      }
      L.prp.swap(qrp);
      L.pci.swap(qci);
    };
    // P^T (by coarse column): rows i and P entry indices, rows ascending
    auto transpose_p = [&]() {
      L.ptp.assign(na + 1, 0);
      for (size_t e = 0; e < L.pci.size(); ++e) ++L.ptp[L.pci[e] + 1];
      for (int I = 0; I < na; ++I) L.ptp[I + 1] += L.ptp[I];
      L.pti.resize(L.pci.size());
      L.pte.resize(L.pci.size());
      std::vector<int32_t> fill(L.ptp.begin(), L.ptp.end() - 1);
      for (int i = 0; i < n; ++i)
        for (int e = L.prp[i]; e < L.prp[i + 1]; ++e) {
          const int32_t q = fill[L.pci[e]]++;
          L.pti[q] = i;
          L.pte[q] = e;
        }
    };
    // the next operator P^T A P would be nearly dense (three-dimensional meshes
    // fill in quickly), counted structurally
    auto too_dense = [&]() {
      std::vector<int32_t> mark(na, -1);
      int64_t cnt = 0;
      for (int I = 0; I < na; ++I)
        for (int k = L.ptp[I]; k < L.ptp[I + 1]; ++k) {
          const int i = L.pti[k];
          for (int e = rp[i]; e < rp[i + 1]; ++e)
            for (int pe = L.prp[ci[e]]; pe < L.prp[ci[e] + 1]; ++pe)
              if (mark[L.pci[pe]] != I) {
                mark[L.pci[pe]] = I;
                ++cnt;
              }
        }
      return cnt > (int64_t)kAmgMaxRowNnz * na;
    };
    // the most smoothing steps (<= p_steps) that keep the next operator below
    // the density bound; if even one step does not, this level becomes the
    // coarsest (Jacobi sweeps, or the dense inverse when small)
    L.np1 = 0;
    bool dense = true;
    if (p_steps == 2) {
      const std::vector<int32_t> prp1 = L.prp, pci1 = L.pci;
      second_step();
      transpose_p();
      dense = too_dense();
      if (dense) {  // back to one step
        L.prp = prp1;
        L.pci = pci1;
        L.np1 = 0;
        L.p1row.clear();
        L.qpp.clear();
        L.qpa.clear();
        L.qpb.clear();
        L.p2src.clear();
      }
    }
    if (dense) {
      transpose_p();
      dense = too_dense();
    }
    if (dense) {
      AmgHostLevel C;
      C.n = L.n;
      C.nc = 0;
      C.rp.swap(L.rp);
      C.ci.swap(L.ci);
      C.diag.swap(L.diag);
      H->levels.push_back(std::move(C));
      break;
    }
    // B = A P : pattern + pairs (A entry, P entry)
    L.brp.assign(1, 0);
    for (int i = 0; i < n; ++i) {
      for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        for (int pe = L.prp[j]; pe < L.prp[j + 1]; ++pe) rg.add(L.pci[pe], e, pe);
      }
      rg.flush(L.bci, L.bpp, L.bpa, &L.bpb);
      L.brp.push_back((int32_t)L.bci.size());
    }
    L.bpp.push_back((int32_t)L.bpa.size());
    // B^T (by coarse column): rows i and B entry indices, rows ascending
    L.btp.assign(na + 1, 0);
    for (size_t e = 0; e < L.bci.size(); ++e) ++L.btp[L.bci[e] + 1];
    for (int I = 0; I < na; ++I) L.btp[I + 1] += L.btp[I];
    L.bti.resize(L.bci.size());
    L.bte.resize(L.bci.size());
    {
      std::vector<int32_t> fill(L.btp.begin(), L.btp.end() - 1);
      for (int i = 0; i < n; ++i)
        for (int e = L.brp[i]; e < L.brp[i + 1]; ++e) {
          const int32_t q = fill[L.bci[e]]++;
          L.bti[q] = i;
          L.bte[q] = e;
        }
    }
    // A_next = P^T B : pattern + pairs (P entry, B entry)
    std::vector<int32_t> nrp(1, 0), nci;
    for (int I = 0; I < na; ++I) {
      for (int k = L.ptp[I]; k < L.ptp[I + 1]; ++k) {
        const int i = L.pti[k], pe = L.pte[k];
        for (int be = L.brp[i]; be < L.brp[i + 1]; ++be) rg.add(L.bci[be], pe, be);
      }
      rg.flush(nci, L.cpp, L.cpa, &L.cpb);
      nrp.push_back((int32_t)nci.size());
    }
    L.cpp.push_back((int32_t)L.cpa.size());
    // next aggregation graph: aggregates adjacent when any of their members are
    {
      std::vector<int32_t> ngp(1, 0), ngi, dummy;
      std::vector<std::vector<int32_t>> members(na);
      for (int i = 0; i < n; ++i) members[L.agg[i]].push_back(i);
      for (int I = 0; I < na; ++I) {
        for (int i : members[I])
          for (int e = grp[i]; e < grp[i + 1]; ++e) rg.add(L.agg[gci[e]], 0, 0);
        std::vector<int32_t> pp;
        rg.flush(ngi, pp, dummy, nullptr);
        dummy.clear();
        ngp.push_back((int32_t)ngi.size());
      }
      grp.swap(ngp);
      gci.swap(ngi);
    }
    H->levels.push_back(std::move(L));
    rp = nrp;
    ci = nci;
    n = na;
  }
}

}  // namespace hho
