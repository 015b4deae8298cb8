// Host-side symbolic analysis: nested-dissection ordering, elimination tree, postorder,
// exact column counts, fundamental + relaxed supernodes, front index lists, relative
// indices for the child->parent extend-add, and the storage plan of the numeric phase.
// The reordering is computed once per pattern and reused (Sec. 3.2-3.3 of the paper).
#include "symbolic.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace gmrf {

namespace {

// ------------------------------------------------------------------ nested dissection
struct NDState {
  int64_t n;
  const int64_t* rp;
  const int32_t* ci;
  const double* X;
  int dim;
  int32_t leaf;
  std::vector<int32_t> stamp;   // membership stamp of the current node set
  std::vector<int8_t> side;     // scratch side labels
  std::vector<int32_t> dist;    // BFS scratch
  int32_t cur = 0;
  std::vector<int32_t> order;
};

// connected components of `nodes` (stamp must mark them with st)
static void components(NDState& S, const std::vector<int32_t>& nodes, int32_t st,
                       std::vector<std::vector<int32_t>>& comps) {
  // visited: stamp becomes st+1
  const int32_t vis = st + 1;
  for (int32_t s0 : nodes) {
    if (S.stamp[s0] != st) continue;
    comps.emplace_back();
    auto& c = comps.back();
    c.push_back(s0);
    S.stamp[s0] = vis;
    for (size_t h = 0; h < c.size(); ++h) {
      int32_t v = c[h];
      for (int64_t e = S.rp[v]; e < S.rp[v + 1]; ++e) {
        int32_t u = S.ci[e];
        if (S.stamp[u] == st) { S.stamp[u] = vis; c.push_back(u); }
      }
    }
  }
}

// BFS levels from root within stamp==st; returns levels' node lists
static void bfs_levels(NDState& S, int32_t root, int32_t st,
                       std::vector<int32_t>& order, std::vector<int32_t>& lvl_ptr) {
  order.clear(); lvl_ptr.clear();
  const int32_t vis = st + 1;
  order.push_back(root); S.stamp[root] = vis;
  lvl_ptr.push_back(0);
  size_t head = 0;
  while (head < order.size()) {
    size_t end = order.size();
    lvl_ptr.push_back((int32_t)end);
    for (; head < end; ++head) {
      int32_t v = order[head];
      for (int64_t e = S.rp[v]; e < S.rp[v + 1]; ++e) {
        int32_t u = S.ci[e];
        if (S.stamp[u] == st) { S.stamp[u] = vis; order.push_back(u); }
      }
    }
  }
  // restore the stamp for reuse by the caller
  for (int32_t v : order) S.stamp[v] = st;
  if (lvl_ptr.back() != (int32_t)order.size()) lvl_ptr.push_back((int32_t)order.size());
}

static void nd_rec(NDState& S, std::vector<int32_t> nodes);

static void emit(NDState& S, const std::vector<int32_t>& nodes) {
  S.order.insert(S.order.end(), nodes.begin(), nodes.end());
}

// Try a coordinate split along axis a; returns separator size or -1.
static int64_t coord_split(NDState& S, const std::vector<int32_t>& nodes, int32_t st, int a,
                           std::vector<int32_t>& A, std::vector<int32_t>& B,
                           std::vector<int32_t>& sep) {
  const size_t m = nodes.size();
  std::vector<double> xs(m);
  for (size_t i = 0; i < m; ++i) xs[i] = S.X[(int64_t)nodes[i] * S.dim + a];
  std::vector<double> tmp(xs);
  std::nth_element(tmp.begin(), tmp.begin() + (m - 1) / 2, tmp.end());
  double med = tmp[(m - 1) / 2];
  size_t nlo = 0;
  for (size_t i = 0; i < m; ++i) nlo += xs[i] <= med;
  if (nlo == m) {  // everything at or below the median: split strictly below instead
    nlo = 0;
    for (size_t i = 0; i < m; ++i) nlo += xs[i] < med;
    if (nlo == 0) return -1;
    for (size_t i = 0; i < m; ++i) S.side[nodes[i]] = xs[i] < med ? 1 : 2;
  } else {
    for (size_t i = 0; i < m; ++i) S.side[nodes[i]] = xs[i] <= med ? 1 : 2;
  }
  // boundary of each side
  std::vector<int32_t> blo, bhi;
  for (size_t i = 0; i < m; ++i) {
    int32_t v = nodes[i];
    int8_t sv = S.side[v];
    for (int64_t e = S.rp[v]; e < S.rp[v + 1]; ++e) {
      int32_t u = S.ci[e];
      if (S.stamp[u] == st && S.side[u] != sv) { (sv == 1 ? blo : bhi).push_back(v); break; }
    }
  }
  const int8_t sepside = blo.size() <= bhi.size() ? 1 : 2;
  std::vector<int32_t>& bs = sepside == 1 ? blo : bhi;
  A.clear(); B.clear(); sep.clear();
  for (int32_t v : bs) S.side[v] = 3;
  for (size_t i = 0; i < m; ++i) {
    int32_t v = nodes[i];
    if (S.side[v] == 1) A.push_back(v);
    else if (S.side[v] == 2) B.push_back(v);
    else sep.push_back(v);
  }
  for (size_t i = 0; i < m; ++i) S.side[nodes[i]] = 0;
  return (int64_t)sep.size();
}

static bool graph_split(NDState& S, const std::vector<int32_t>& nodes, int32_t st,
                        std::vector<int32_t>& A, std::vector<int32_t>& B,
                        std::vector<int32_t>& sep) {
  std::vector<int32_t> order, lp;
  // pseudo-peripheral root: two sweeps
  int32_t root = nodes[0];
  for (int it = 0; it < 2; ++it) {
    bfs_levels(S, root, st, order, lp);
    root = order.back();
  }
  bfs_levels(S, root, st, order, lp);
  const int nl = (int)lp.size() - 1;
  if (nl < 3) return false;
  const size_t half = order.size() / 2;
  int best = -1;
  for (int l = 1; l < nl - 1; ++l) {
    if ((size_t)lp[l + 1] > half) { best = l; break; }
  }
  if (best < 1) best = nl / 2;
  A.assign(order.begin(), order.begin() + lp[best]);
  sep.assign(order.begin() + lp[best], order.begin() + lp[best + 1]);
  B.assign(order.begin() + lp[best + 1], order.end());
  return !A.empty() && !B.empty();
}

static void nd_rec(NDState& S, std::vector<int32_t> nodes) {
  if ((int32_t)nodes.size() <= S.leaf) { emit(S, nodes); return; }
  S.cur += 2;
  const int32_t st = S.cur;
  for (int32_t v : nodes) S.stamp[v] = st;
  std::vector<std::vector<int32_t>> comps;
  components(S, nodes, st, comps);
  if (comps.size() > 1) {
    for (auto& c : comps) nd_rec(S, std::move(c));
    return;
  }
  for (int32_t v : nodes) S.stamp[v] = st;   // components() moved them to st+1
  std::vector<int32_t> A, B, sep;
  bool ok = false;
  if (S.X) {
    int64_t best = -1;
    std::vector<int32_t> a2, b2, s2;
    for (int a = 0; a < S.dim; ++a) {
      int64_t sz = coord_split(S, nodes, st, a, a2, b2, s2);
      if (sz < 0 || a2.empty() || b2.empty()) continue;
      // prefer the smallest separator; break ties towards balance
      int64_t imb = std::llabs((int64_t)a2.size() - (int64_t)b2.size());
      int64_t bimb = std::llabs((int64_t)A.size() - (int64_t)B.size());
      if (best < 0 || sz < best || (sz == best && imb < bimb)) {
        best = sz; A.swap(a2); B.swap(b2); sep.swap(s2);
      }
    }
    ok = best >= 0;
  }
  if (!ok) ok = graph_split(S, nodes, st, A, B, sep);
  if (!ok) { emit(S, nodes); return; }
  nodes.clear(); nodes.shrink_to_fit();
  nd_rec(S, std::move(A));
  nd_rec(S, std::move(B));
  emit(S, sep);
}

}  // namespace

void nested_dissection(int64_t n, const int64_t* rp, const int32_t* ci, const double* coords,
                       int dim, int32_t leaf, std::vector<int32_t>& perm) {
  NDState S;
  S.n = n; S.rp = rp; S.ci = ci; S.X = coords; S.dim = dim; S.leaf = std::max(leaf, 1);
  S.stamp.assign(n, 0);
  S.side.assign(n, 0);
  S.order.reserve(n);
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  nd_rec(S, std::move(all));
  perm.swap(S.order);
}

// ------------------------------------------------------------------ etree / postorder
void elimination_tree(int64_t n, const int64_t* rp, const int32_t* ci,
                      const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
                      std::vector<int32_t>& parent) {
  parent.assign(n, -1);
  std::vector<int32_t> anc(n, -1);
  for (int64_t j = 0; j < n; ++j) {
    const int32_t o = perm[j];
    for (int64_t e = rp[o]; e < rp[o + 1]; ++e) {
      int32_t r = iperm[ci[e]];
      if (r >= j) continue;
      // climb from r to the root of its current subtree, compressing towards j
      while (anc[r] != -1 && anc[r] != j) {
        int32_t t = anc[r];
        anc[r] = (int32_t)j;
        r = t;
      }
      if (anc[r] == -1) { anc[r] = (int32_t)j; parent[r] = (int32_t)j; }
    }
  }
}

static void postorder(int64_t n, const std::vector<int32_t>& parent, std::vector<int32_t>& post) {
  std::vector<int32_t> head(n, -1), next(n, -1), stack;
  for (int64_t j = n - 1; j >= 0; --j) {
    if (parent[j] >= 0) { next[j] = head[parent[j]]; head[parent[j]] = (int32_t)j; }
  }
  post.clear(); post.reserve(n);
  for (int64_t r = 0; r < n; ++r) {
    if (parent[r] != -1) continue;
    stack.push_back((int32_t)r);
    while (!stack.empty()) {
      int32_t v = stack.back();
      int32_t c = head[v];
      if (c == -1) { stack.pop_back(); post.push_back(v); }
      else { head[v] = next[c]; stack.push_back(c); }
    }
  }
}

// Column counts from the row subtrees of the elimination tree (Gilbert, Ng and Peyton):
// row i of L has a nonzero in column j iff j lies on a path from some k (A_ik != 0,
// k < i) up to i.  Counting leaves of each row subtree with a least-common-ancestor
// correction gives every column count in near-linear time.  Requires a postordered tree.
void column_counts(int64_t n, const int64_t* rp, const int32_t* ci,
                   const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
                   const std::vector<int32_t>& parent, std::vector<int64_t>& cc) {
  std::vector<int32_t> first(n, -1), maxfirst(n, -1), prevleaf(n, -1), anc(n);
  std::vector<int64_t> delta(n, 0);
  for (int64_t k = 0; k < n; ++k) {
    int32_t j = (int32_t)k;
    delta[j] = (first[j] == -1) ? 1 : 0;          // leaf of the etree
    for (; j != -1 && first[j] == -1; j = parent[j]) first[j] = (int32_t)k;
  }
  for (int64_t i = 0; i < n; ++i) anc[i] = (int32_t)i;
  for (int64_t k = 0; k < n; ++k) {
    const int32_t j = (int32_t)k;
    if (parent[j] != -1) delta[parent[j]]--;
    const int32_t o = perm[j];
    for (int64_t e = rp[o]; e < rp[o + 1]; ++e) {
      const int32_t i = iperm[ci[e]];
      if (i <= j || first[j] <= maxfirst[i]) continue;   // j is not a leaf of row i's subtree
      maxfirst[i] = first[j];
      const int32_t jprev = prevleaf[i];
      prevleaf[i] = j;
      delta[j]++;
      if (jprev != -1) {
        int32_t q = jprev;
        while (q != anc[q]) q = anc[q];
        for (int32_t s = jprev, sp; s != q; s = sp) { sp = anc[s]; anc[s] = q; }
        delta[q]--;                                         // overlap counted twice
      }
    }
    if (parent[j] != -1) anc[j] = parent[j];
  }
  cc.assign(delta.begin(), delta.end());
  for (int64_t j = 0; j < n; ++j)
    if (parent[j] != -1) cc[parent[j]] += cc[j];
}

// ------------------------------------------------------------------ full analysis
std::string analyze(int64_t n, const int64_t* rp, const int32_t* ci, const double* coords,
                    int dim, const AnalyzeOptions& opt, Symbolic& out, const int32_t* perm_in) {
  if (n <= 0) return "matrix dimension must be positive";
  if (n >= (int64_t)1 << 31) return "dimension exceeds 2^31-1";
  Symbolic& Y = out;
  Y = Symbolic();
  Y.n = n;
  // 1. ordering: nested dissection, or the caller's order (postordered below either way)
  std::vector<int32_t> perm0;
  if (perm_in) {
    perm0.assign(perm_in, perm_in + n);
    std::vector<char> seen(n, 0);
    for (int64_t k = 0; k < n; ++k) {
      const int32_t o = perm0[k];
      if (o < 0 || o >= n || seen[o]) return "the given order is not a permutation";
      seen[o] = 1;
    }
  } else {
    nested_dissection(n, rp, ci, coords, dim, opt.leaf_size, perm0);
  }
  if ((int64_t)perm0.size() != n) return "internal: ordering lost nodes";
  std::vector<int32_t> ip0(n);
  for (int64_t k = 0; k < n; ++k) ip0[perm0[k]] = (int32_t)k;
  // 2. etree + postorder, then re-derive everything in postordered numbering
  std::vector<int32_t> par0, post;
  elimination_tree(n, rp, ci, perm0, ip0, par0);
  postorder(n, par0, post);
  Y.perm.resize(n);
  for (int64_t k = 0; k < n; ++k) Y.perm[k] = perm0[post[k]];
  Y.iperm.resize(n);
  for (int64_t k = 0; k < n; ++k) Y.iperm[Y.perm[k]] = (int32_t)k;
  elimination_tree(n, rp, ci, Y.perm, Y.iperm, Y.parent);
  column_counts(n, rp, ci, Y.perm, Y.iperm, Y.parent, Y.colcount);
  Y.nnzL = 0;
  double f = 0.0;
  for (int64_t j = 0; j < n; ++j) { Y.nnzL += Y.colcount[j]; f += (double)Y.colcount[j] * (double)Y.colcount[j]; }
  Y.flops_factor = f;
  Y.flops_selinv = 2.0 * f;
  Y.flops_solve = 4.0 * (double)Y.nnzL - 2.0 * (double)n;

  // 3. fundamental supernodes
  std::vector<int32_t> nchild(n, 0);
  for (int64_t j = 0; j < n; ++j) if (Y.parent[j] >= 0) nchild[Y.parent[j]]++;
  std::vector<int32_t> fs;  // fundamental supernode starts
  fs.push_back(0);
  for (int64_t j = 1; j < n; ++j) {
    bool same = Y.parent[j - 1] == j && Y.colcount[j - 1] == Y.colcount[j] + 1 && nchild[j] == 1;
    if (!same) fs.push_back((int32_t)j);
  }
  const int32_t nf = (int32_t)fs.size();
  fs.push_back((int32_t)n);
  std::vector<int32_t> fsup(n);
  for (int32_t s = 0; s < nf; ++s)
    for (int32_t j = fs[s]; j < fs[s + 1]; ++j) fsup[j] = s;
  std::vector<int32_t> fpar(nf, -1);
  for (int32_t s = 0; s < nf; ++s) {
    int32_t pj = Y.parent[fs[s + 1] - 1];
    fpar[s] = pj >= 0 ? fsup[pj] : -1;
  }

  // 4. relaxed amalgamation: merge the last child (columns adjacent) into its parent
  struct Node { int32_t first, p; int64_t nfront; double exact; int32_t top; };
  std::vector<int32_t> rep(nf);
  std::iota(rep.begin(), rep.end(), 0);
  auto find = [&](int32_t x) {
    while (rep[x] != x) { rep[x] = rep[rep[x]]; x = rep[x]; }
    return x;
  };
  std::vector<Node> st;
  for (int32_t s = 0; s < nf; ++s) {
    Node cur;
    cur.first = fs[s]; cur.p = fs[s + 1] - fs[s];
    cur.nfront = Y.colcount[fs[s]];
    cur.exact = 0;
    for (int32_t j = fs[s]; j < fs[s + 1]; ++j) cur.exact += (double)Y.colcount[j];
    cur.top = s;
    while (!st.empty()) {
      const Node& c = st.back();
      if (c.first + c.p != cur.first) break;
      int32_t cp = fpar[c.top];
      if (cp < 0 || find(cp) != s) break;
      const int64_t p = (int64_t)c.p + cur.p;
      const int64_t nfr = (int64_t)c.p + cur.nfront;
      const double stored = (double)p * (double)nfr - 0.5 * (double)p * (double)(p - 1);
      const double zeros = stored - (c.exact + cur.exact);
      const double frac = zeros / stored;
      bool merge = p <= opt.relax_small ||
                   (p <= opt.relax_mid && frac <= opt.relax_frac_mid) ||
                   (p <= opt.relax_big && frac <= opt.relax_frac_big) ||
                   frac <= opt.relax_frac_any;
      if (!merge) break;
      rep[c.top] = s;
      cur.first = c.first; cur.p = (int32_t)p; cur.nfront = nfr; cur.exact += c.exact;
      st.pop_back();
    }
    st.push_back(cur);
  }
  // representative of every fundamental supernode after merging -> final index
  Y.ns = (int32_t)st.size();
  std::vector<int32_t> fin_of_top(nf, -1);
  for (int32_t s = 0; s < Y.ns; ++s) fin_of_top[st[s].top] = s;
  Y.sfirst.resize(Y.ns + 1);
  for (int32_t s = 0; s < Y.ns; ++s) Y.sfirst[s] = st[s].first;
  Y.sfirst[Y.ns] = (int32_t)n;
  std::vector<int32_t> colsup(n);
  for (int32_t s = 0; s < Y.ns; ++s)
    for (int32_t j = Y.sfirst[s]; j < Y.sfirst[s + 1]; ++j) colsup[j] = s;
  Y.sparent.assign(Y.ns, -1);
  for (int32_t s = 0; s < Y.ns; ++s) {
    int32_t pj = Y.parent[Y.sfirst[s + 1] - 1];
    Y.sparent[s] = pj >= 0 ? colsup[pj] : -1;
    if (Y.sparent[s] >= 0 && Y.sparent[s] <= s) return "internal: supernode tree not postordered";
  }
  // children CSR
  Y.child_ptr.assign(Y.ns + 1, 0);
  for (int32_t s = 0; s < Y.ns; ++s) if (Y.sparent[s] >= 0) Y.child_ptr[Y.sparent[s] + 1]++;
  for (int32_t s = 0; s < Y.ns; ++s) Y.child_ptr[s + 1] += Y.child_ptr[s];
  Y.child_idx.assign(Y.child_ptr[Y.ns], 0);
  {
    std::vector<int32_t> fill(Y.child_ptr.begin(), Y.child_ptr.end() - 1);
    for (int32_t s = 0; s < Y.ns; ++s) if (Y.sparent[s] >= 0) Y.child_idx[fill[Y.sparent[s]]++] = s;
  }

  // 5. front index lists F_s = S_s u R_s
  Y.rowptr.assign(Y.ns + 1, 0);
  std::vector<std::vector<int32_t>> R(Y.ns);
  std::vector<int32_t> mark(n, -1);
  for (int32_t s = 0; s < Y.ns; ++s) {
    const int32_t f0 = Y.sfirst[s], f1 = Y.sfirst[s + 1];
    std::vector<int32_t>& r = R[s];
    for (int32_t j = f0; j < f1; ++j) {
      const int32_t o = Y.perm[j];
      for (int64_t e = rp[o]; e < rp[o + 1]; ++e) {
        int32_t i = Y.iperm[ci[e]];
        if (i >= f1 && mark[i] != s) { mark[i] = s; r.push_back(i); }
      }
    }
    for (int32_t t = Y.child_ptr[s]; t < Y.child_ptr[s + 1]; ++t) {
      for (int32_t i : R[Y.child_idx[t]])
        if (i >= f1 && mark[i] != s) { mark[i] = s; r.push_back(i); }
    }
    std::sort(r.begin(), r.end());
    Y.rowptr[s + 1] = Y.rowptr[s] + (f1 - f0) + (int64_t)r.size();
    // children's R lists are no longer needed once the parent is built; keep them for
    // the relative-index pass below (memory: sum of u_s ints)
  }
  Y.rows.resize(Y.rowptr[Y.ns]);
  Y.relpos.assign(Y.rowptr[Y.ns], -1);
  for (int32_t s = 0; s < Y.ns; ++s) {
    int64_t o = Y.rowptr[s];
    for (int32_t j = Y.sfirst[s]; j < Y.sfirst[s + 1]; ++j) Y.rows[o++] = j;
    for (int32_t i : R[s]) Y.rows[o++] = i;
  }
  R.clear(); R.shrink_to_fit();
  // relative indices child R -> parent front
  for (int32_t s = 0; s < Y.ns; ++s) {
    const int32_t par = Y.sparent[s];
    if (par < 0) {
      if (Y.nf(s) != Y.p(s)) return "internal: root supernode with rows below";
      continue;
    }
    const int32_t* pr = &Y.rows[Y.rowptr[par]];
    const int32_t pn = Y.nf(par);
    int32_t q = 0;
    for (int64_t e = Y.rowptr[s] + Y.p(s); e < Y.rowptr[s + 1]; ++e) {
      const int32_t i = Y.rows[e];
      while (q < pn && pr[q] < i) ++q;
      if (q >= pn || pr[q] != i) return "internal: child row missing from parent front";
      Y.relpos[e] = q;
    }
  }
  // 6. depths, storage
  Y.depth.assign(Y.ns, 0);
  Y.max_depth = 0;
  for (int32_t s = Y.ns - 1; s >= 0; --s) {
    Y.depth[s] = Y.sparent[s] >= 0 ? Y.depth[Y.sparent[s]] + 1 : 0;
    Y.max_depth = std::max(Y.max_depth, Y.depth[s]);
  }
  Y.Loff.assign(Y.ns, 0);
  Y.Doff.assign(Y.ns, 0);
  Y.Woff.assign(Y.ns, 0);
  Y.Voff.assign(Y.ns, 0);
  std::vector<int64_t> wlev(Y.max_depth + 1, 0), vlev(Y.max_depth + 1, 0);
  int64_t L = 0, D = 0;
  Y.stored_L = 0;
  for (int32_t s = 0; s < Y.ns; ++s) {
    const int64_t p = Y.p(s), nfr = Y.nf(s);
    Y.Loff[s] = L;
    L += nfr * p;
    Y.stored_L += nfr * p - p * (p - 1) / 2;
    Y.Doff[s] = D;
    D += ((p + opt.nb - 1) / opt.nb) * (int64_t)opt.nb * opt.nb;
    const int d = Y.depth[s];
    Y.Woff[s] = wlev[d];
    wlev[d] += nfr * nfr;
    Y.Voff[s] = vlev[d];
    vlev[d] += nfr;
  }
  Y.Lsize = L;
  Y.Dsize = D;
  for (int d = 0; d <= Y.max_depth; ++d) {
    Y.Wsize[d & 1] = std::max(Y.Wsize[d & 1], wlev[d]);
    Y.Vsize[d & 1] = std::max(Y.Vsize[d & 1], vlev[d]);
  }
  return std::string();
}

}  // namespace gmrf
