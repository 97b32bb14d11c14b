// Symbolic phase of the coarsest level's sparse direct solver (nested
// dissection, fronts, index maps); see direct.h for the ordering and the
// numeric scheme.  Depends on the mesh topology and the level's layout only.
#include <algorithm>
#include <cstdlib>
#include <numeric>
#include <string>

#include "direct.h"

namespace hho {
namespace {

struct Node {
  int32_t lo, hi;              // cells perm[lo, hi)
  int32_t c[2] = {-1, -1};
  int32_t parent = -1, depth = 0;
};

struct Sets {  // disjoint sets of cells with path halving
  std::vector<int32_t> up;
  explicit Sets(int n) : up(n) { std::iota(up.begin(), up.end(), 0); }
  int32_t find(int32_t a) {
    while (up[a] != a) {
      up[a] = up[up[a]];
      a = up[a];
    }
    return a;
  }
  void join(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) up[std::max(a, b)] = std::min(a, b);
  }
};

}  // namespace

void nd_symbolic(const hho_mesh *mesh, int d, int p, int t, int cond, bool pin, const std::vector<int32_t> &rowptr,
                 const std::vector<int32_t> &col, const std::vector<int64_t> &seg_cell_ptr, NdHost *H) {
  const int nc = (int)mesh->nc, nf = (int)mesh->nf;
  const int dp = d * p;
  const int64_t nface = (int64_t)nf * dp;
  const int bs = cond == HHO_COND_V ? p : dp;
  if (pin && t != 1) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: a pressure null space needs t = 1");
  if (nface + (int64_t)nc * t > INT32_MAX)  // unknowns are stored as 32-bit indices
    fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: more than 2^31 - 1 coarse unknowns");
  *H = NdHost{};
  // members (a batch's disjoint problems; one problem: all cells)
  if (seg_cell_ptr.empty())
    H->segp = {0, (int64_t)nc};
  else
    H->segp = seg_cell_ptr;
  const int nsegp = (int)H->segp.size() - 1;
  H->cseg.assign(nc, 0);
  for (int s = 0; s < nsegp; ++s)
    for (int64_t c = H->segp[s]; c < H->segp[s + 1]; ++c) H->cseg[c] = s;
  H->pins.assign(nsegp, -1);

  // ---- nested dissection of the cells: a node holding cells of several members
  // (disjoint problems, cells numbered member by member) is split between
  // members, near the middle, at no cost; within one member, recursive
  // coordinate bisection at the median of the cell centres along the longest
  // side of their bounding box
  std::vector<int32_t> perm(nc);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<Node> nodes;
  nodes.push_back(Node{0, nc});
  for (size_t k = 0; k < nodes.size(); ++k) {
    const int32_t lo = nodes[k].lo, hi = nodes[k].hi;
    const int32_t s0 = H->cseg[perm[lo]], s1 = H->cseg[perm[hi - 1]];
    if (s0 != s1) {  // perm is still the identity here: members are contiguous ranges
      int32_t best = -1;
      for (int32_t s = s0 + 1; s <= s1; ++s) {
        const int32_t b = (int32_t)H->segp[s];
        if (best < 0 || std::abs(2 * b - lo - hi) < std::abs(2 * best - lo - hi)) best = b;
      }
      const int32_t depth = nodes[k].depth + 1;
      for (int c = 0; c < 2; ++c) {
        Node ch{c == 0 ? lo : best, c == 0 ? best : hi};
        ch.parent = (int32_t)k;
        ch.depth = depth;
        nodes[k].c[c] = (int32_t)nodes.size();
        nodes.push_back(ch);
      }
      continue;
    }
    if (hi - lo <= kNdLeafCells) continue;
    double bl[3] = {1e300, 1e300, 1e300}, bh[3] = {-1e300, -1e300, -1e300};
    for (int32_t i = lo; i < hi; ++i)
      for (int a = 0; a < 3; ++a) {
        const double x = mesh->ccen[3 * (size_t)perm[i] + a];
        bl[a] = std::min(bl[a], x);
        bh[a] = std::max(bh[a], x);
      }
    int ax = 0;
    for (int a = 1; a < mesh->dim; ++a)
      if (bh[a] - bl[a] > bh[ax] - bl[ax]) ax = a;
    const int32_t mid = lo + (hi - lo) / 2;
    std::nth_element(perm.begin() + lo, perm.begin() + mid, perm.begin() + hi, [&](int32_t x, int32_t y) {
      const double u = mesh->ccen[3 * (size_t)x + ax], v = mesh->ccen[3 * (size_t)y + ax];
      return u < v || (u == v && x < y);
    });
    const int32_t depth = nodes[k].depth + 1;
    for (int s = 0; s < 2; ++s) {
      Node c{s == 0 ? lo : mid, s == 0 ? mid : hi};
      c.parent = (int32_t)k;
      c.depth = depth;
      nodes[k].c[s] = (int32_t)nodes.size();
      nodes.push_back(c);
    }
  }
  const int nn = (int)nodes.size();
  std::vector<int32_t> leaf_of(nc, -1);
  for (int k = 0; k < nn; ++k)
    if (nodes[k].c[0] < 0)
      for (int32_t i = nodes[k].lo; i < nodes[k].hi; ++i) leaf_of[perm[i]] = k;
  // postorder (children before parents, each subtree contiguous)
  std::vector<int32_t> post;
  post.reserve(nn);
  {
    std::vector<std::pair<int32_t, int>> st{{0, 0}};
    while (!st.empty()) {
      auto &top = st.back();
      const int32_t k = top.first;
      if (top.second < 2 && nodes[k].c[top.second] >= 0) {
        const int32_t c = nodes[k].c[top.second++];
        st.push_back({c, 0});
      } else {
        post.push_back(k);
        st.pop_back();
      }
    }
  }
  std::vector<int32_t> rank_of(nn);
  for (int i = 0; i < nn; ++i) rank_of[post[i]] = i;

  // ---- faces: the node where the face's cells are separated
  auto lca = [&](int32_t a, int32_t b) {
    while (nodes[a].depth > nodes[b].depth) a = nodes[a].parent;
    while (nodes[b].depth > nodes[a].depth) b = nodes[b].parent;
    while (a != b) {
      a = nodes[a].parent;
      b = nodes[b].parent;
    }
    return a;
  };
  std::vector<std::vector<int32_t>> fs_faces(nn), placed(nn), delayed(nn);
  for (int f = 0; f < nf; ++f) {
    const int64_t c0 = mesh->fcell[0][f], c1 = mesh->fcell[1][f];
    const int32_t k = c1 < 0 ? leaf_of[c0] : lca(leaf_of[c0], leaf_of[c1]);
    fs_faces[k].push_back(f);
  }

  // ---- pressures: within each set of cells connected through eliminated faces,
  // all but one are eliminated at the node; the last is passed up
  Sets sets(nc);
  std::vector<int32_t> last_of(nc, -1);
  std::vector<int32_t> pinned_cells;
  for (int i = 0; i < nn; ++i) {
    const int32_t k = post[i];
    for (int32_t f : fs_faces[k]) {
      const int64_t c1 = mesh->fcell[1][f];
      if (c1 >= 0) sets.join((int32_t)mesh->fcell[0][f], (int32_t)c1);
    }
    std::vector<int32_t> cand;
    if (nodes[k].c[0] < 0) {
      cand.assign(perm.begin() + nodes[k].lo, perm.begin() + nodes[k].hi);
      std::sort(cand.begin(), cand.end());
    } else {
      for (int s = 0; s < 2; ++s)
        cand.insert(cand.end(), delayed[nodes[k].c[s]].begin(), delayed[nodes[k].c[s]].end());
    }
    for (int32_t c : cand) last_of[sets.find(c)] = c;
    for (int32_t c : cand) (last_of[sets.find(c)] == c ? delayed[k] : placed[k]).push_back(c);
    for (int32_t c : cand) last_of[sets.find(c)] = -1;
    if (k == 0) {  // root: one pressure left per connected set of cells
      if (pin) {  // each must be one member's null space
        for (int32_t c : delayed[0]) {
          int64_t &slot = H->pins[H->cseg[c]];
          if (slot >= 0)
            fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: the mesh of a problem with a pressure null space "
                                    "must be connected");
          slot = nface + (int64_t)c * t;
        }
        for (int64_t v : H->pins)
          if (v < 0) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: a member without its null space");
        pinned_cells = delayed[0];
      } else {
        placed[0].insert(placed[0].end(), delayed[0].begin(), delayed[0].end());
      }
      delayed[0].clear();
    }
  }

  // ---- unknown groups (face f: f; cell T: nf + T), their front and elimination key
  const int ng = nf + nc;
  std::vector<int32_t> gfront(ng, -1);   // postorder rank of the front eliminating the group
  std::vector<int64_t> gkey(ng, INT64_MAX);  // elimination key of the group's first unknown
  std::vector<std::vector<int32_t>> fsg(nn);
  int64_t key = 0;
  auto gsize = [&](int32_t g) { return g < nf ? dp : t; };
  for (int i = 0; i < nn; ++i) {
    const int32_t k = post[i];
    std::sort(fs_faces[k].begin(), fs_faces[k].end());
    for (int32_t f : fs_faces[k]) fsg[i].push_back(f);
    for (int32_t c : placed[k]) fsg[i].push_back(nf + c);
    for (int32_t g : fsg[i]) {
      gfront[g] = i;
      gkey[g] = key;
      key += gsize(g);
    }
  }
  for (int32_t c : pinned_cells) gfront[nf + c] = -1;

  // ---- update sets (groups adjacent to the subtree, eliminated above it), by front rank
  std::vector<std::vector<int32_t>> upg(nn);
  std::vector<int32_t> stamp(ng, -1);
  std::vector<int32_t> rank_children(2 * (size_t)nn, -1);
  for (int i = 0; i < nn; ++i) {
    const int32_t k = post[i];
    for (int s = 0; s < 2; ++s)
      if (nodes[k].c[s] >= 0) rank_children[2 * i + s] = rank_of[nodes[k].c[s]];
  }
  for (int i = 0; i < nn; ++i) {
    std::vector<int32_t> &S = upg[i];
    auto add = [&](int32_t g) {
      if (stamp[g] == i || gfront[g] <= i) return;  // already in, pinned (-1) or eliminated in the subtree
      stamp[g] = i;
      S.push_back(g);
    };
    for (int s = 0; s < 2; ++s)
      if (rank_children[2 * i + s] >= 0)
        for (int32_t g : upg[rank_children[2 * i + s]]) add(g);
    for (int32_t g : fsg[i]) {
      if (g < nf) {
        for (int s = 0; s < 2; ++s) {
          const int64_t c = mesh->fcell[s][g];
          if (c < 0) continue;
          add(nf + (int32_t)c);
          for (int64_t e = mesh->cptr[c]; e < mesh->cptr[c + 1]; ++e) add((int32_t)mesh->cface[e]);
        }
      } else {
        const int32_t c = g - nf;
        for (int64_t e = mesh->cptr[c]; e < mesh->cptr[c + 1]; ++e) add((int32_t)mesh->cface[e]);
      }
    }
    std::sort(S.begin(), S.end(), [&](int32_t a, int32_t b) { return gkey[a] < gkey[b]; });
  }

  // ---- fronts: unknown lists, sizes, offsets
  auto gdof0 = [&](int32_t g) { return g < nf ? (int64_t)g * dp : nface + (int64_t)(g - nf) * t; };
  std::vector<int64_t> ekey(nface + (int64_t)nc * t, INT64_MAX);  // elimination key of every unknown
  for (int32_t g = 0; g < ng; ++g)
    if (gfront[g] >= 0)
      for (int q = 0; q < gsize(g); ++q) ekey[gdof0(g) + q] = gkey[g] + q;
  H->nfront = nn;
  H->m.resize(nn);
  H->nfs.resize(nn);
  H->off.assign(nn + 1, 0);
  H->voff.assign(nn + 1, 0);
  H->dofoff.assign(nn + 1, 0);
  H->child.assign(rank_children.begin(), rank_children.end());
  std::vector<int64_t> kbeg(nn);
  for (int i = 0; i < nn; ++i) {
    int64_t a = 0, b = 0;
    for (int32_t g : fsg[i]) a += gsize(g);
    for (int32_t g : upg[i]) b += gsize(g);
    if (a + b > (int64_t)1 << 20) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: front too large");
    H->nfs[i] = (int32_t)a;
    H->m[i] = (int32_t)(a + b);
    H->maxm = std::max(H->maxm, H->m[i]);
    kbeg[i] = fsg[i].empty() ? 0 : gkey[fsg[i][0]];
    H->off[i + 1] = H->off[i] + (int64_t)H->m[i] * H->m[i];
    H->voff[i + 1] = H->voff[i] + H->m[i];
    H->dofoff[i + 1] = H->dofoff[i] + H->m[i];
    H->factor_entries += (int64_t)H->m[i] * H->m[i] - b * b;
    for (int32_t g : fsg[i])
      for (int q = 0; q < gsize(g); ++q) H->dof.push_back((int32_t)(gdof0(g) + q));
    for (int32_t g : upg[i])
      for (int q = 0; q < gsize(g); ++q) H->dof.push_back((int32_t)(gdof0(g) + q));
  }
  H->total = H->off[nn];
  H->vtotal = H->voff[nn];
  // position of unknown j in front i (j eliminated in i or above it)
  auto pos_in = [&](int i, int64_t j) -> int32_t {
    const int64_t kj = ekey[j];
    if (kj >= kbeg[i] && kj < kbeg[i] + H->nfs[i]) return (int32_t)(kj - kbeg[i]);
    const int32_t *u = H->dof.data() + H->dofoff[i] + H->nfs[i];
    const int n = H->m[i] - H->nfs[i];
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (ekey[u[mid]] < kj) lo = mid + 1; else hi = mid;
    }
    return (lo < n && u[lo] == j) ? H->nfs[i] + lo : -1;
  };
  // child maps: position of each front unknown in a child's update part
  H->cmap.assign(2 * (size_t)H->dofoff[nn], -1);
  for (int i = 0; i < nn; ++i)
    for (int s = 0; s < 2; ++s) {
      const int32_t c = H->child[2 * i + s];
      if (c < 0) continue;
      int64_t found = 0;
      for (int32_t a = 0; a < H->m[i]; ++a) {
        const int32_t pc = pos_in(c, H->dof[H->dofoff[i] + a]);
        if (pc >= 0 && pc >= H->nfs[c]) {
          H->cmap[2 * (H->dofoff[i] + a) + s] = pc - H->nfs[c];
          ++found;
        }
      }
      if (found != H->m[c] - H->nfs[c]) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: inconsistent fronts");
    }

  // ---- where each operator entry lands: the front of the earlier-eliminated unknown
  auto place = [&](int64_t src, int64_t i, int64_t j) {
    if (ekey[i] == INT64_MAX || ekey[j] == INT64_MAX) return;  // the pinned unknown
    const int64_t first = ekey[i] < ekey[j] ? i : j;
    int fr = -1;
    {  // front of `first`: the group's front
      const int32_t g = first < nface ? (int32_t)(first / dp) : nf + (int32_t)((first - nface) / t);
      fr = gfront[g];
    }
    const int32_t a = pos_in(fr, i), b = pos_in(fr, j);
    if (a < 0 || b < 0) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: entry outside its front");
    H->src.push_back(src);
    H->dst.push_back(H->off[fr] + (int64_t)a * H->m[fr] + b);
  };
  const int64_t nnzb = rowptr[nf];
  int64_t src = 0;
  for (int f = 0; f < nf; ++f)
    for (int32_t b = rowptr[f]; b < rowptr[f + 1]; ++b) {
      const int g = col[b];
      for (int rr = 0; rr < bs; ++rr)
        for (int cc = 0; cc < bs; ++cc, ++src) {
          if (cond == HHO_COND_V) {
            for (int c = 0; c < d; ++c)
              place(src, ((int64_t)f * d + c) * p + rr, ((int64_t)g * d + c) * p + cc);
          } else {
            place(src, (int64_t)f * bs + rr, (int64_t)g * bs + cc);
          }
        }
    }
  if (src != nnzb * bs * bs) fail(HHO_E_INVALID_ARG, "sparse direct coarse solver: block count");
  for (int c = 0; c < nc; ++c)
    for (int64_t e = mesh->cptr[c]; e < mesh->cptr[c + 1]; ++e) {
      const int64_t f = mesh->cface[e];
      for (int cr = 0; cr < dp; ++cr)
        for (int q = 0; q < t; ++q, ++src) {
          const int64_t rf = f * dp + cr, cT = nface + (int64_t)c * t + q;
          place(src, rf, cT);
          place(src, cT, rf);
        }
    }
  if (cond == HHO_COND_V)
    for (int c = 0; c < nc; ++c)
      for (int q = 0; q < t; ++q)
        for (int q2 = 0; q2 < t; ++q2, ++src)
          place(src, nface + (int64_t)c * t + q, nface + (int64_t)c * t + q2);

  // ---- heights, and the launch tables of each height
  std::vector<int32_t> height(nn, 0);
  for (int i = 0; i < nn; ++i)
    for (int s = 0; s < 2; ++s)
      if (H->child[2 * i + s] >= 0) height[i] = std::max(height[i], height[H->child[2 * i + s]] + 1);
  H->nheight = *std::max_element(height.begin(), height.end()) + 1;
  H->hptr.assign(H->nheight + 1, 0);
  for (int i = 0; i < nn; ++i) ++H->hptr[height[i] + 1];
  for (int h = 0; h < H->nheight; ++h) H->hptr[h + 1] += H->hptr[h];
  H->hfront.resize(nn);
  {
    std::vector<int32_t> at(H->hptr.begin(), H->hptr.end() - 1);
    for (int i = 0; i < nn; ++i) H->hfront[at[height[i]]++] = i;
  }
  H->big.assign(H->nheight, 0);
  H->hmaxnfs.assign(H->nheight, 0);
  H->hmaxm.assign(H->nheight, 0);
  H->soff.assign(nn, 0);
  H->tptr.assign(H->nheight + 1, 0);
  H->cptr.assign(H->nheight + 1, 0);
  H->scptr.assign(H->nheight + 1, 0);
  for (int h = 0; h < H->nheight; ++h) {
    int64_t scratch = 0;
    for (int32_t x = H->hptr[h]; x < H->hptr[h + 1]; ++x) {
      const int i = H->hfront[x];
      H->hmaxnfs[h] = std::max(H->hmaxnfs[h], H->nfs[i]);
      H->hmaxm[h] = std::max(H->hmaxm[h], H->m[i]);
    }
    H->big[h] = H->hmaxm[h] > kNdSmall;
    for (int32_t x = H->hptr[h]; x < H->hptr[h + 1]; ++x) {
      const int i = H->hfront[x];
      const int m = H->m[i];
      for (int r = 0; r < m; r += kNdChunk) {
        H->chunks.push_back(i);
        H->chunks.push_back(r);
      }
      for (int r = 0; r < m; r += kNdSolveRows) {
        H->schunks.push_back(i);
        H->schunks.push_back(r);
      }
      if (H->big[h]) {
        H->soff[i] = scratch;
        scratch += (int64_t)kNdPanel * kNdPanel + 2 * (int64_t)m * kNdPanel;
        for (int r = 0; r < m; r += kNdTile)
          for (int c = 0; c <= r; c += kNdTile) {  // lower triangle; the kernels mirror the rest
            H->tiles.push_back(i);
            H->tiles.push_back(r);
            H->tiles.push_back(c);
          }
      }
    }
    H->stotal = std::max(H->stotal, scratch);
    H->tptr[h + 1] = (int32_t)(H->tiles.size() / 3);
    H->cptr[h + 1] = (int32_t)(H->chunks.size() / 2);
    H->scptr[h + 1] = (int32_t)(H->schunks.size() / 2);
  }
}

}  // namespace hho
