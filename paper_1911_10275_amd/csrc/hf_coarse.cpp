// Host-side structure of the two-level preconditioner (symbolic work only:
// index sets, orderings and maps; every number is computed on the device).
//
// Coarse space.  One P1 vertex function per "vertex class": the copies of a
// mesh vertex in the elements around it (each element carries its own
// discontinuous nodes) are merged across every intact interface (all points
// in state 0, no fluid) and kept apart across a crack or cohesive face, so
// the coarse functions are continuous where the solid is intact and may
// jump where it is cracked.  Copies of clamped vertices get no class.  The
// prolongation P maps class values to the element nodes with the P1 weights
// of the node positions (1 at the vertex, 1/2 at the edge midpoints);
// clamped node copies get 0.
//
// Coarse solver.  A_c = P^T A P is factorised by a multifrontal Gauss-Jordan
// elimination on a nested-dissection tree of the classes: recursive
// coordinate bisection along the longest extent, with the classes of the
// lower half that touch the upper half as the separator.  Every tree node
// owns a set of classes (a leaf block or a separator) and a front (its own
// classes followed by the ancestors' classes its subtree couples to); the
// fronts are eliminated level by level from the leaves.
#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <vector>

#include "hf_internal.h"

namespace hf {

namespace {

struct Dsu {
  std::vector<int64_t> p;
  explicit Dsu(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int64_t find(int64_t x) {
    while (p[x] != x) {
      p[x] = p[p[x]];
      x = p[x];
    }
    return x;
  }
  void unite(int64_t a, int64_t b) {
    a = find(a);
    b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

struct NdNode {
  std::vector<int32_t> own;       // classes eliminated here (sorted)
  std::vector<int32_t> children;  // tree node ids
};

// nested dissection of the classes in `ids` (modified); returns the node id
int nd_build(std::vector<int32_t> ids, const std::vector<double> &xyz, int dim,
             const std::vector<int64_t> &adj_ptr, const std::vector<int32_t> &adj,
             std::vector<int8_t> &side, int leaf_max, std::vector<NdNode> &nodes) {
  const int me = (int)nodes.size();
  nodes.emplace_back();
  if ((int)ids.size() <= leaf_max) {
    std::sort(ids.begin(), ids.end());
    nodes[me].own = ids;
    return me;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t c : ids)
    for (int d = 0; d < dim; ++d) {
      lo[d] = std::min(lo[d], xyz[(int64_t)c * dim + d]);
      hi[d] = std::max(hi[d], xyz[(int64_t)c * dim + d]);
    }
  int ax = 0;
  for (int d = 1; d < dim; ++d)
    if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
  std::sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
    const double xa = xyz[(int64_t)a * dim + ax], xb = xyz[(int64_t)b * dim + ax];
    return xa != xb ? xa < xb : a < b;
  });
  // split at the widest gap of the sorted coordinates within the middle
  // fifth (on a layered mesh this cuts between two layers instead of
  // through one, which would thicken the separator)
  const size_t n = ids.size();
  size_t mid = n / 2;
  {
    const size_t lo = std::max<size_t>(1, (size_t)(0.4 * n)), hi = std::min(n - 1, (size_t)(0.6 * n) + 1);
    double best = -1.0;
    for (size_t i = lo; i <= hi; ++i) {
      const double gap = xyz[(int64_t)ids[i] * dim + ax] - xyz[(int64_t)ids[i - 1] * dim + ax];
      if (gap > best) {
        best = gap;
        mid = i;
      }
    }
  }
  for (size_t i = 0; i < ids.size(); ++i) side[ids[i]] = i < mid ? 0 : 1;
  std::vector<int32_t> left, right, sep;
  for (size_t i = 0; i < ids.size(); ++i) {
    const int32_t c = ids[i];
    if (i >= mid) {
      right.push_back(c);
      continue;
    }
    bool touches = false;
    for (int64_t q = adj_ptr[c]; q < adj_ptr[c + 1] && !touches; ++q) touches = side[adj[q]] == 1;
    (touches ? sep : left).push_back(c);
  }
  for (int32_t c : ids) side[c] = -1;
  std::sort(sep.begin(), sep.end());
  nodes[me].own = sep;
  std::vector<int32_t> ch;
  if (!left.empty()) ch.push_back(nd_build(std::move(left), xyz, dim, adj_ptr, adj, side, leaf_max, nodes));
  if (!right.empty()) ch.push_back(nd_build(std::move(right), xyz, dim, adj_ptr, adj, side, leaf_max, nodes));
  nodes[me].children = ch;
  return me;
}

}  // namespace

// P1 weights of the element nodes: for local vertex v, the nodes a with a
// non-zero weight and the weights (vertex node 1, edge midpoints 1/2)
int vertex_node_weights(int dim, int order, int v, int *nodes, double *w) {
  static const int E2[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  static const int E3[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
  int n = 0;
  nodes[n] = v;
  w[n++] = 1.0;
  if (order == 2) {
    const int ne = dim == 2 ? 3 : 6;
    for (int k = 0; k < ne; ++k) {
      const int *ed = dim == 2 ? E2[k] : E3[k];
      if (ed[0] == v || ed[1] == v) {
        nodes[n] = dim + 1 + k;
        w[n++] = 0.5;
      }
    }
  }
  return n;
}

void build_coarse_plan(const CoarseIn &in, CoarsePlan &cp) {
  const int dim = in.dim, NV = dim + 1, NQ = in.nq, NN = in.nn;
  const int64_t ne = in.ne;
  cp = CoarsePlan{};
  cp.dim = dim;
  cp.nv = NV;
  // ---- vertex classes ------------------------------------------------------
  Dsu dsu(ne * NV);
  for (int64_t f = 0; f < in.nf; ++f) {
    bool intact = in.beta[f] == 0;
    for (int q = 0; q < NQ && intact; ++q) intact = in.qp_state[f * NQ + q] == 0;
    if (!intact) continue;
    for (int k = 0; k < dim; ++k)
      dsu.unite((int64_t)in.face_em[f] * NV + in.fperm_m[f * dim + k],
                (int64_t)in.face_ep[f] * NV + in.fperm_p[f * dim + k]);
  }
  cp.cls_of.assign(ne * NV, -1);
  std::vector<int64_t> root_cls(ne * NV, -1);
  cp.coff.assign(in.n_inst + 1, 0);
  int32_t ncls = 0;
  for (int b = 0; b < in.n_inst; ++b) {
    for (int64_t e = in.eoff[b]; e < in.eoff[b + 1]; ++e)
      for (int v = 0; v < NV; ++v) {
        if (in.clamp[e] & (1u << (v * dim))) continue;  // a clamped vertex node: no class
        const int64_t r = dsu.find(e * NV + v);
        if (root_cls[r] < 0) {
          root_cls[r] = ncls++;
          const int32_t vert = in.elem[e * NV + v];
          for (int d = 0; d < dim; ++d) cp.xyz.push_back(in.xyz[(int64_t)vert * dim + d]);
          cp.cinst.push_back(b);
        }
        cp.cls_of[e * NV + v] = (int32_t)root_cls[r];
      }
    cp.coff[b + 1] = ncls;
  }
  cp.ncls = ncls;
  // restriction lists: the copies of each class
  cp.rc_ptr.assign(ncls + 1, 0);
  for (int64_t x = 0; x < ne * NV; ++x)
    if (cp.cls_of[x] >= 0) cp.rc_ptr[cp.cls_of[x] + 1]++;
  for (int32_t c = 0; c < ncls; ++c) cp.rc_ptr[c + 1] += cp.rc_ptr[c];
  cp.rc_list.assign(cp.rc_ptr[ncls], 0);
  {
    std::vector<int32_t> fill(cp.rc_ptr.begin(), cp.rc_ptr.end() - 1);
    for (int64_t x = 0; x < ne * NV; ++x)
      if (cp.cls_of[x] >= 0) cp.rc_list[fill[cp.cls_of[x]]++] = (int32_t)x;
  }
  // ---- columns of A P per element row: the classes of its block columns ----
  cp.ap_ptr.assign(ne + 1, 0);
  for (int64_t e = 0; e < ne; ++e) {
    std::vector<int32_t> cols;
    for (int64_t k = in.blk_ptr[e]; k < in.blk_ptr[e + 1]; ++k) {
      const int64_t f = in.blk_col[k];
      for (int v = 0; v < NV; ++v)
        if (cp.cls_of[f * NV + v] >= 0) cols.push_back(cp.cls_of[f * NV + v]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    cp.ap_cls.insert(cp.ap_cls.end(), cols.begin(), cols.end());
    cp.ap_ptr[e + 1] = (int64_t)cp.ap_cls.size();
    cp.max_ap = std::max<int>(cp.max_ap, (int)cols.size());
  }
  // ---- coupled class pairs of A_c and their contributions -------------------
  struct Contrib {
    int32_t ci, cj, e;
    int16_t v, j;
  };
  // Pattern of A_c: the pairs of classes that share an element, plus the
  // pairs across interfaces that are not intact (kept apart in the coarse
  // space): a class of a vertex of such a face with every class of the
  // neighbour.  Any other pair (cI, cJ) gets contributions only through
  // faces that do not contain cI's vertex, whose face integrals vanish with
  // e's test functions there, so it is an exact zero.  Pairs in the
  // pattern keep every contribution: those through an intact face from the
  // two sides cancel only together.
  std::vector<int64_t> pat;
  for (int64_t e = 0; e < ne; ++e)
    for (int v = 0; v < NV; ++v) {
      const int32_t ci = cp.cls_of[e * NV + v];
      if (ci < 0) continue;
      for (int w = 0; w < NV; ++w)
        if (cp.cls_of[e * NV + w] >= 0) pat.push_back((int64_t)ci * ncls + cp.cls_of[e * NV + w]);
      for (int lf = 0; lf < NV; ++lf) {
        if (lf == v) continue;  // the face opposite v does not contain it
        const int64_t f = in.nbr[e * NV + lf];
        if (f < 0) continue;
        bool intact = true;  // the face's classes are shared across it
        for (int w = 0; w < NV && intact; ++w) {
          if (w == lf) continue;
          const int32_t g = in.elem[e * NV + w];
          for (int w2 = 0; w2 < NV; ++w2)
            if (in.elem[f * NV + w2] == g && cp.cls_of[f * NV + w2] != cp.cls_of[e * NV + w]) intact = false;
        }
        if (intact) continue;
        for (int w2 = 0; w2 < NV; ++w2)
          if (cp.cls_of[f * NV + w2] >= 0) pat.push_back((int64_t)ci * ncls + cp.cls_of[f * NV + w2]);
      }
    }
  std::sort(pat.begin(), pat.end());
  pat.erase(std::unique(pat.begin(), pat.end()), pat.end());
  std::vector<Contrib> con;
  con.reserve((size_t)ne * NV * 8);
  for (int64_t e = 0; e < ne; ++e)
    for (int v = 0; v < NV; ++v) {
      const int32_t ci = cp.cls_of[e * NV + v];
      if (ci < 0) continue;
      for (int64_t j = cp.ap_ptr[e]; j < cp.ap_ptr[e + 1]; ++j) {
        const int32_t cj = cp.ap_cls[j];
        if (!std::binary_search(pat.begin(), pat.end(), (int64_t)ci * ncls + cj)) continue;
        con.push_back({ci, cj, (int32_t)e, (int16_t)v, (int16_t)(j - cp.ap_ptr[e])});
      }
    }
  std::sort(con.begin(), con.end(), [](const Contrib &a, const Contrib &b) {
    if (a.ci != b.ci) return a.ci < b.ci;
    if (a.cj != b.cj) return a.cj < b.cj;
    if (a.e != b.e) return a.e < b.e;
    return a.v < b.v;
  });
  std::vector<int32_t> pair_i, pair_j;
  cp.pair_cptr.push_back(0);
  for (size_t t = 0; t < con.size(); ++t) {
    if (t == 0 || con[t].ci != con[t - 1].ci || con[t].cj != con[t - 1].cj) {
      if (t) cp.pair_cptr.push_back((int64_t)t);
      pair_i.push_back(con[t].ci);
      pair_j.push_back(con[t].cj);
    }
    cp.pc_e.push_back(con[t].e);
    cp.pc_vj.push_back((int32_t)con[t].v | ((int32_t)con[t].j << 8));
  }
  cp.pair_cptr.push_back((int64_t)con.size());
  const int64_t npair = (int64_t)pair_i.size();
  con.clear();
  con.shrink_to_fit();
  // class adjacency (symmetrised pattern of A_c)
  std::vector<int64_t> adj_ptr(ncls + 1, 0);
  std::vector<int32_t> adj;
  {
    std::vector<std::vector<int32_t>> nb(ncls);
    for (int64_t p = 0; p < npair; ++p)
      if (pair_i[p] != pair_j[p]) {
        nb[pair_i[p]].push_back(pair_j[p]);
        nb[pair_j[p]].push_back(pair_i[p]);
      }
    for (int32_t c = 0; c < ncls; ++c) {
      auto &v = nb[c];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      adj.insert(adj.end(), v.begin(), v.end());
      adj_ptr[c + 1] = (int64_t)adj.size();
    }
  }
  // ---- nested dissection per instance (a forest) ----------------------------
  std::vector<NdNode> nodes;
  std::vector<int8_t> side(ncls, -1);
  std::vector<int> roots;
  for (int b = 0; b < in.n_inst; ++b) {
    std::vector<int32_t> ids;
    for (int32_t c = cp.coff[b]; c < cp.coff[b + 1]; ++c) ids.push_back(c);
    if (ids.empty()) continue;
    roots.push_back(nd_build(std::move(ids), cp.xyz, dim, adj_ptr, adj, side, in.leaf_max, nodes));
  }
  const int nn = (int)nodes.size();
  // post order: elimination order of the classes, heights
  std::vector<int> post, height(nn, 0), parent(nn, -1);
  {
    std::vector<std::pair<int, int>> stk;
    for (int r : roots) {
      stk.push_back({r, 0});
      while (!stk.empty()) {
        auto &[x, i] = stk.back();
        if (i < (int)nodes[x].children.size()) {
          const int c = nodes[x].children[i++];
          parent[c] = x;
          stk.push_back({c, 0});
        } else {
          for (int c : nodes[x].children) height[x] = std::max(height[x], height[c] + 1);
          post.push_back(x);
          stk.pop_back();
        }
      }
    }
  }
  std::vector<int64_t> order(ncls, -1);
  std::vector<int> owner(ncls, -1);
  {
    int64_t o = 0;
    for (int x : post)
      for (int32_t c : nodes[x].own) {
        order[c] = o++;
        owner[c] = x;
      }
  }
  // symbolic factorisation: fronts (own classes, then ancestor classes the
  // subtree couples to, by elimination order)
  std::vector<std::vector<int32_t>> front(nn);
  std::vector<int> kcls(nn, 0);
  for (int x : post) {
    const NdNode &nd = nodes[x];
    // every class outside the subtree that the subtree couples to belongs to
    // an ancestor (nested dissection), i.e. comes later in the order than
    // all of the node's own classes; with no own classes (an empty
    // separator) the children's struct classes are all ancestors
    int64_t maxo = -1;
    for (int32_t c : nd.own) maxo = std::max(maxo, order[c]);
    std::vector<int32_t> st;
    for (int32_t c : nd.own)
      for (int64_t q = adj_ptr[c]; q < adj_ptr[c + 1]; ++q)
        if (order[adj[q]] > maxo) st.push_back(adj[q]);
    for (int ch : nd.children)
      for (size_t t = kcls[ch]; t < front[ch].size(); ++t)
        if (order[front[ch][t]] > maxo) st.push_back(front[ch][t]);
    std::sort(st.begin(), st.end(), [&](int32_t a, int32_t b) { return order[a] < order[b]; });
    st.erase(std::unique(st.begin(), st.end()), st.end());
    std::vector<int32_t> fl = nd.own;
    fl.insert(fl.end(), st.begin(), st.end());
    kcls[x] = (int)nd.own.size();
    front[x] = std::move(fl);
  }
  // ---- levels (by height) and device layout of the fronts -------------------
  int nlev = 0;
  for (int x = 0; x < nn; ++x) nlev = std::max(nlev, height[x] + 1);
  cp.n_nodes = nn;
  cp.n_levels = nlev;
  cp.level_ptr.assign(nlev + 1, 0);
  for (int x = 0; x < nn; ++x) cp.level_ptr[height[x] + 1]++;
  for (int l = 0; l < nlev; ++l) cp.level_ptr[l + 1] += cp.level_ptr[l];
  cp.level_nodes.assign(nn, 0);
  {
    std::vector<int32_t> fill(cp.level_ptr.begin(), cp.level_ptr.end() - 1);
    // nodes of a level in tree order (post order), so the layout is fixed
    for (int x : post) cp.level_nodes[fill[height[x]]++] = x;
  }
  cp.fk.assign(nn, 0);
  cp.ff.assign(nn, 0);
  cp.fo.assign(nn, 0);
  cp.uo.assign(nn, 0);
  cp.fd_ptr.assign(nn + 1, 0);
  cp.level_maxk.assign(nlev, 0);
  cp.level_maxf.assign(nlev, 0);
  int64_t fo = 0, uo = 0;
  // fronts stored level by level
  for (int l = 0; l < nlev; ++l)
    for (int32_t t = cp.level_ptr[l]; t < cp.level_ptr[l + 1]; ++t) {
      const int x = cp.level_nodes[t];
      const int f = (int)front[x].size() * dim, k = kcls[x] * dim;
      cp.fk[x] = k;
      cp.ff[x] = f;
      cp.fo[x] = fo;
      fo += (int64_t)f * f;
      cp.uo[x] = uo;
      uo += f - k;
      cp.level_maxk[l] = std::max(cp.level_maxk[l], k);
      cp.level_maxf[l] = std::max(cp.level_maxf[l], f);
    }
  cp.front_total = fo;
  cp.upd_total = uo;
  for (int x = 0; x < nn; ++x) cp.fd_ptr[x + 1] = cp.fd_ptr[x] + cp.ff[x];
  // global coarse DOF of every front position, and where the children's
  // update rows land (at most two sources per position)
  cp.fd_dof.assign(cp.fd_ptr[nn], 0);
  cp.src0.assign(cp.fd_ptr[nn], -1);
  cp.src1.assign(cp.fd_ptr[nn], -1);
  std::vector<int64_t> cpos(ncls, -1);
  for (int x = 0; x < nn; ++x) {
    for (size_t t = 0; t < front[x].size(); ++t)
      for (int i = 0; i < dim; ++i) cp.fd_dof[cp.fd_ptr[x] + t * dim + i] = front[x][t] * dim + i;
  }
  cp.ea_ptr.assign(nn + 1, 0);
  cp.child_slot.assign(nn, -1);
  cp.parent.assign(nn, -1);
  for (int x = 0; x < nn; ++x) {
    cp.parent[x] = parent[x];
    for (size_t s = 0; s < nodes[x].children.size(); ++s) cp.child_slot[nodes[x].children[s]] = (int32_t)s;
  }
  for (int x = 0; x < nn; ++x) {
    // positions of this node's front classes
    for (size_t t = 0; t < front[x].size(); ++t) cpos[front[x][t]] = (int64_t)t;
    for (size_t s = 0; s < nodes[x].children.size(); ++s) {
      const int ch = nodes[x].children[s];
      for (size_t t = kcls[ch]; t < front[ch].size(); ++t) {
        const int64_t pos = cpos[front[ch][t]];
        if (pos < 0) throw std::runtime_error("coarse symbolic: child struct class missing in parent front");
        for (int i = 0; i < dim; ++i) {
          const int64_t d = cp.fd_ptr[x] + pos * dim + i;
          const int64_t srow = cp.uo[ch] + (int64_t)(t - kcls[ch]) * dim + i;
          if (cp.src0[d] < 0) cp.src0[d] = srow;
          else if (cp.src1[d] < 0) cp.src1[d] = srow;
          else throw std::runtime_error("coarse symbolic: more than two children");
        }
      }
    }
    for (size_t t = 0; t < front[x].size(); ++t) cpos[front[x][t]] = -1;
  }
  // extend-add maps (class level): child struct entry -> parent front position
  for (int x = 0; x < nn; ++x) {
    const int pa = parent[x];
    if (pa >= 0) {
      for (size_t t = 0; t < front[pa].size(); ++t) cpos[front[pa][t]] = (int64_t)t;
      for (size_t t = kcls[x]; t < front[x].size(); ++t) cp.ea_map.push_back((int32_t)cpos[front[x][t]]);
      for (size_t t = 0; t < front[pa].size(); ++t) cpos[front[pa][t]] = -1;
    }
    cp.ea_ptr[x + 1] = (int64_t)cp.ea_map.size();
  }
  // destination of every class pair in the front of the node that
  // eliminates its earlier class
  cp.pair_dest.assign(npair, 0);
  cp.pair_ld.assign(npair, 0);
  {
    std::vector<std::vector<int64_t>> by_node(nn);
    for (int64_t p = 0; p < npair; ++p) {
      const int32_t a = pair_i[p], b = pair_j[p];
      by_node[order[a] < order[b] ? owner[a] : owner[b]].push_back(p);
    }
    for (int x = 0; x < nn; ++x) {
      for (size_t t = 0; t < front[x].size(); ++t) cpos[front[x][t]] = (int64_t)t;
      for (int64_t p : by_node[x]) {
        const int64_t pa = cpos[pair_i[p]], pb = cpos[pair_j[p]];
        if (pa < 0 || pb < 0) throw std::runtime_error("coarse symbolic: pair outside its front");
        cp.pair_dest[p] = cp.fo[x] + pa * dim * cp.ff[x] + pb * dim;
        cp.pair_ld[p] = cp.ff[x];
      }
      for (size_t t = 0; t < front[x].size(); ++t) cpos[front[x][t]] = -1;
    }
  }
  cp.n_pairs = npair;
  // GJ flop count (for reporting)
  double fl = 0.0;
  for (int x = 0; x < nn; ++x) fl += 2.0 * (double)cp.ff[x] * cp.ff[x] * cp.fk[x];
  cp.factor_flops = fl;
}

}  // namespace hf
