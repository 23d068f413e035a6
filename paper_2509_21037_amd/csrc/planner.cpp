// Host planner: nested-dissection ordering, symbolic factorisation with
// relaxed supernodes, numeric supernodal Cholesky (FP64) and the staircase
// plan of the Schur-complement assembly.
#include "planner.hpp"
#include "dense_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

namespace scasm {

namespace {

// ---------------------------------------------------------------------------
// node graph (K's pattern compressed by DOFs per node)
// ---------------------------------------------------------------------------
struct Graph {
    int32_t nv = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
};

Graph node_graph(const SubdomainInput& in) {
    const int32_t dpn = in.dofs_per_node;
    Graph g;
    g.nv = in.n / dpn;
    std::vector<std::vector<int32_t>> nb(g.nv);
    for (int32_t r = 0; r < in.n; ++r) {
        const int32_t u = r / dpn;
        for (int64_t p = in.rowptr[r]; p < in.rowptr[r + 1]; ++p) {
            const int32_t v = in.col[p] / dpn;
            if (v != u) nb[u].push_back(v);
        }
    }
    g.ptr.assign(g.nv + 1, 0);
    for (int32_t u = 0; u < g.nv; ++u) {
        auto& v = nb[u];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        g.ptr[u + 1] = g.ptr[u] + (int64_t)v.size();
    }
    g.adj.resize(g.ptr[g.nv]);
    for (int32_t u = 0; u < g.nv; ++u)
        std::copy(nb[u].begin(), nb[u].end(), g.adj.begin() + g.ptr[u]);
    return g;
}

// ---------------------------------------------------------------------------
// nested dissection: order(A), order(B), then the separator S.  With node
// coordinates the split is the middle plane (among the distinct coordinate
// values) of the axis of largest extent; without them it is the middle BFS
// level from a pseudo-peripheral node.  Any edge left between A and B moves
// its B end into S, so S always separates.
// ---------------------------------------------------------------------------
class Dissector {
public:
    Dissector(const Graph& g, const double* coords, int dim, int leaf)
        : g_(g), coords_(coords), dim_(dim), leaf_(std::max(1, leaf)),
          side_(g.nv, -1), stamp_(g.nv, 0), level_(g.nv, -1) {}

    void run(std::vector<int32_t>& order) {
        std::vector<int32_t> all(g_.nv);
        std::iota(all.begin(), all.end(), 0);
        order.clear();
        order.reserve(g_.nv);
        dissect(all, order);
    }

private:
    const Graph& g_;
    const double* coords_;
    int dim_, leaf_;
    std::vector<int8_t> side_;
    std::vector<int32_t> stamp_;
    std::vector<int32_t> level_;
    int32_t tick_ = 0;

    void dissect(std::vector<int32_t>& sub, std::vector<int32_t>& order) {
        if ((int)sub.size() <= leaf_) {
            std::sort(sub.begin(), sub.end());
            order.insert(order.end(), sub.begin(), sub.end());
            return;
        }
        std::vector<int32_t> A, B, S;
        bool ok = coords_ ? split_plane(sub, A, B, S) : split_bfs(sub, A, B, S);
        if (!ok || S.size() == sub.size()) {
            std::sort(sub.begin(), sub.end());
            order.insert(order.end(), sub.begin(), sub.end());
            return;
        }
        fix_separator(A, B, S);
        std::vector<int32_t>().swap(sub);
        dissect(A, order);
        dissect(B, order);
        std::sort(S.begin(), S.end());
        order.insert(order.end(), S.begin(), S.end());
    }

    bool split_plane(const std::vector<int32_t>& sub, std::vector<int32_t>& A,
                     std::vector<int32_t>& B, std::vector<int32_t>& S) {
        int axis = -1;
        double best = 0;
        for (int d = 0; d < dim_; ++d) {
            double lo = coords_[(size_t)sub[0] * dim_ + d], hi = lo;
            for (int32_t v : sub) {
                const double x = coords_[(size_t)v * dim_ + d];
                lo = std::min(lo, x);
                hi = std::max(hi, x);
            }
            if (hi - lo > best) { best = hi - lo; axis = d; }
        }
        if (axis < 0) return false;
        std::vector<double> vals;
        vals.reserve(sub.size());
        for (int32_t v : sub) vals.push_back(coords_[(size_t)v * dim_ + axis]);
        std::sort(vals.begin(), vals.end());
        vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        const double plane = vals[(vals.size() - 1) / 2];
        for (int32_t v : sub) {
            const double x = coords_[(size_t)v * dim_ + axis];
            if (x < plane) A.push_back(v);
            else if (x > plane) B.push_back(v);
            else S.push_back(v);
        }
        return true;
    }

    bool split_bfs(const std::vector<int32_t>& sub, std::vector<int32_t>& A,
                   std::vector<int32_t>& B, std::vector<int32_t>& S) {
        ++tick_;
        for (int32_t v : sub) stamp_[v] = tick_;
        int32_t root = sub[0];
        int32_t depth = 0;
        std::vector<int32_t> q;
        for (int it = 0; it < 4; ++it) {          // pseudo-peripheral node search
            int32_t far = bfs(root, q, depth);
            if (it > 0 && level_[far] <= depth && far == root) break;
            if (it == 3) break;
            root = far;
        }
        bfs(root, q, depth);
        if (depth < 2) return false;
        const int32_t mid = depth / 2;
        std::vector<int8_t> seen(0);
        for (int32_t v : sub) {
            const int32_t lv = level_[v];
            if (lv < 0) B.push_back(v);           // other components
            else if (lv < mid) A.push_back(v);
            else if (lv > mid) B.push_back(v);
            else S.push_back(v);
        }
        return true;
    }

    // BFS restricted to the current subset; fills level_, returns the last node.
    int32_t bfs(int32_t root, std::vector<int32_t>& q, int32_t& depth) {
        q.clear();
        for (int32_t i = 0; i < (int32_t)level_.size(); ++i)
            if (stamp_[i] == tick_) level_[i] = -1;
        level_[root] = 0;
        q.push_back(root);
        size_t h = 0;
        int32_t last = root;
        while (h < q.size()) {
            const int32_t u = q[h++];
            last = u;
            for (int64_t p = g_.ptr[u]; p < g_.ptr[u + 1]; ++p) {
                const int32_t v = g_.adj[p];
                if (stamp_[v] == tick_ && level_[v] < 0) {
                    level_[v] = level_[u] + 1;
                    q.push_back(v);
                }
            }
        }
        depth = level_[last];
        return last;
    }

    void fix_separator(std::vector<int32_t>& A, std::vector<int32_t>& B, std::vector<int32_t>& S) {
        for (int32_t v : A) side_[v] = 0;
        for (int32_t v : B) side_[v] = 1;
        for (int32_t v : S) side_[v] = 2;
        for (int32_t a : A)
            for (int64_t p = g_.ptr[a]; p < g_.ptr[a + 1]; ++p) {
                const int32_t b = g_.adj[p];
                if (side_[b] == 1) side_[b] = 2;
            }
        std::vector<int32_t> B2;
        for (int32_t b : B) {
            if (side_[b] == 2) S.push_back(b);
            else B2.push_back(b);
        }
        B.swap(B2);
        for (int32_t v : A) side_[v] = -1;
        for (int32_t v : B) side_[v] = -1;
        for (int32_t v : S) side_[v] = -1;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
std::string build_plan(const SubdomainInput& in, const PlanOptions& opt, SubPlan& P, int& code) {
    code = 1;
    const int32_t n = in.n;
    if (n <= 0) return "n must be positive";
    if (n >= (1 << 27)) return "n must be below 2^27";
    if (!in.rowptr || !in.col) return "K_reg pattern missing";
    if (in.m < 0) return "m must be non-negative";
    if (in.m > 0 && (!in.dof || !in.sign)) return "B^T columns missing";
    const int32_t dpn = in.dofs_per_node > 0 ? in.dofs_per_node : 1;
    if (n % dpn != 0) return "n is not a multiple of dofs_per_node";
    if (in.rowptr[0] != 0) return "rowptr[0] must be 0";
    for (int32_t r = 0; r < n; ++r) {
        if (in.rowptr[r + 1] < in.rowptr[r]) return "rowptr not monotone";
        for (int64_t p = in.rowptr[r]; p < in.rowptr[r + 1]; ++p)
            if (in.col[p] < 0 || in.col[p] >= n) return "column index out of range";
    }
    for (int32_t j = 0; j < in.m; ++j) {
        if (in.dof[j] < 0 || in.dof[j] >= n) return "B^T dof out of range";
        if (in.sign[j] != 1 && in.sign[j] != -1) return "B^T sign must be +1 or -1";
    }
    if (in.coords && in.dim <= 0) return "coords given without dim";

    P = SubPlan();
    P.n = n;
    P.m = in.m;
    P.dpn = dpn;

    // ---- ordering
    P.perm.resize(n);
    if (in.perm) {
        std::vector<char> seen(n, 0);
        for (int32_t i = 0; i < n; ++i) {
            const int32_t v = in.perm[i];
            if (v < 0 || v >= n || seen[v]) return "perm is not a permutation";
            seen[v] = 1;
            P.perm[i] = v;
        }
    } else {
        Graph g = node_graph(in);
        std::vector<int32_t> norder;
        Dissector d(g, in.coords, in.dim, opt.leaf_nodes);
        d.run(norder);
        for (int32_t k = 0; k < g.nv; ++k)
            for (int32_t c = 0; c < dpn; ++c) P.perm[(size_t)k * dpn + c] = norder[k] * dpn + c;
    }
    P.iperm.resize(n);
    for (int32_t i = 0; i < n; ++i) P.iperm[P.perm[i]] = i;
    const auto& iperm = P.iperm;

    // ---- lower pattern of P K P^T by columns (rows > j)
    std::vector<int64_t> cptr(n + 1, 0);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t i = iperm[r];
        for (int64_t p = in.rowptr[r]; p < in.rowptr[r + 1]; ++p) {
            const int32_t j = iperm[in.col[p]];
            if (i > j) ++cptr[j + 1];
        }
    }
    for (int32_t j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
    std::vector<int32_t> crow(cptr[n]);
    {
        std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
        for (int32_t r = 0; r < n; ++r) {
            const int32_t i = iperm[r];
            for (int64_t p = in.rowptr[r]; p < in.rowptr[r + 1]; ++p) {
                const int32_t j = iperm[in.col[p]];
                if (i > j) crow[fill[j]++] = i;
            }
        }
        for (int32_t j = 0; j < n; ++j) {
            std::sort(crow.begin() + cptr[j], crow.begin() + cptr[j + 1]);
            // duplicates (repeated CSR entries) are harmless for the symbolic
            // phase; they are removed when structures are merged
        }
    }

    // ---- elimination tree (Liu, with path compression) from rows of the lower part
    P.parent.assign(n, -1);
    {
        std::vector<int32_t> anc(n, -1);
        for (int32_t i = 0; i < n; ++i) {          // rows in increasing permuted order
            const int32_t r = P.perm[i];
            for (int64_t p = in.rowptr[r]; p < in.rowptr[r + 1]; ++p) {
                int32_t j = iperm[in.col[p]];
                if (j >= i) continue;
                while (anc[j] != -1 && anc[j] != i) {
                    const int32_t nx = anc[j];
                    anc[j] = i;
                    j = nx;
                }
                if (anc[j] == -1) {
                    anc[j] = i;
                    P.parent[j] = i;
                }
            }
        }
    }
    // the column ordering must be topological for the tree (children < parent);
    // Liu's algorithm guarantees parent[j] > j.

    // ---- exact column structures (counts) by merging children
    std::vector<int32_t> nchild(n, 0);
    std::vector<std::vector<int32_t>> kids(n);
    for (int32_t j = 0; j < n; ++j)
        if (P.parent[j] >= 0) {
            ++nchild[P.parent[j]];
            kids[P.parent[j]].push_back(j);
        }
    P.colcount.assign(n, 0);
    {
        std::vector<std::vector<int32_t>> st(n);
        std::vector<int32_t> mark(n, -1);
        for (int32_t j = 0; j < n; ++j) {
            std::vector<int32_t> s;
            for (int64_t p = cptr[j]; p < cptr[j + 1]; ++p) {
                const int32_t i = crow[p];
                if (mark[i] != j) { mark[i] = j; s.push_back(i); }
            }
            for (int32_t c : kids[j]) {
                for (int32_t i : st[c])
                    if (i > j && mark[i] != j) { mark[i] = j; s.push_back(i); }
                std::vector<int32_t>().swap(st[c]);
            }
            std::sort(s.begin(), s.end());
            P.colcount[j] = 1 + (int32_t)s.size();
            st[j].swap(s);
        }
    }
    P.nnzL = 0;
    for (int32_t j = 0; j < n; ++j) P.nnzL += P.colcount[j];

    // ---- fundamental supernodes
    std::vector<int32_t> fstart;
    for (int32_t j = 0; j < n; ++j) {
        const bool cont = j > 0 && P.parent[j - 1] == j && nchild[j] == 1 &&
                          P.colcount[j - 1] == P.colcount[j] + 1;
        if (!cont) fstart.push_back(j);
    }
    fstart.push_back(n);
    const int32_t nf = (int32_t)fstart.size() - 1;

    // ---- relaxed amalgamation: merge a supernode into its parent when the
    // child ends right before the parent, the merged width stays below
    // relax_width and the explicit zeros stay below relax_zero_frac.
    std::vector<int32_t> fcol2s(n);
    for (int32_t s = 0; s < nf; ++s)
        for (int32_t j = fstart[s]; j < fstart[s + 1]; ++j) fcol2s[j] = s;
    std::vector<int32_t> gstart;          // group starts (in columns)
    {
        // group g covers fundamental supernodes [gfirst, glast]; stats kept per group
        std::vector<int32_t> grp_of(nf);
        std::vector<int64_t> g_exact;
        std::vector<int32_t> g_first_col, g_width;
        for (int32_t s = 0; s < nf; ++s) {
            const int32_t f = fstart[s], w = fstart[s + 1] - f;
            int64_t exact = 0;
            for (int32_t j = f; j < f + w; ++j) exact += P.colcount[j];
            const int32_t r = P.colcount[f] - w;      // rows below the fundamental supernode
            bool merged = false;
            if (s > 0 && !g_first_col.empty()) {
                const int32_t gc = (int32_t)g_first_col.size() - 1;   // group ending at f-1
                const int32_t lastc = f - 1;
                if (P.parent[lastc] >= f && P.parent[lastc] < f + w) {
                    const int64_t W = (int64_t)g_width[gc] + w;
                    const int64_t stored = W * (W + 1) / 2 + W * (int64_t)r;
                    const int64_t ex = g_exact[gc] + exact;
                    const double zf = stored > 0 ? double(stored - ex) / double(stored) : 0.0;
                    if (W <= opt.relax_width && (W <= 4 || zf <= opt.relax_zero_frac)) {
                        g_width[gc] = (int32_t)W;
                        g_exact[gc] = ex;
                        merged = true;
                    }
                }
            }
            if (!merged) {
                g_first_col.push_back(f);
                g_width.push_back(w);
                g_exact.push_back(exact);
            }
        }
        gstart = g_first_col;
        gstart.push_back(n);
    }
    P.nsuper = (int32_t)gstart.size() - 1;
    P.sfirst = gstart;
    P.col2super.resize(n);
    for (int32_t s = 0; s < P.nsuper; ++s)
        for (int32_t j = P.sfirst[s]; j < P.sfirst[s + 1]; ++j) P.col2super[j] = s;

    // ---- supernodal row structures: own columns, then the union of the
    // columns' lower entries and the children's structures below the supernode
    {
        std::vector<std::vector<int32_t>> below(P.nsuper);
        std::vector<std::vector<int32_t>> skids(P.nsuper);
        std::vector<int32_t> mark(n, -1);
        for (int32_t s = 0; s < P.nsuper; ++s) {
            const int32_t f = P.sfirst[s], l = P.sfirst[s + 1] - 1;
            std::vector<int32_t> rows;
            for (int32_t j = f; j <= l; ++j)
                for (int64_t p = cptr[j]; p < cptr[j + 1]; ++p) {
                    const int32_t i = crow[p];
                    if (i > l && mark[i] != s) { mark[i] = s; rows.push_back(i); }
                }
            for (int32_t c : skids[s])
                for (int32_t i : below[c])
                    if (i > l && mark[i] != s) { mark[i] = s; rows.push_back(i); }
            std::sort(rows.begin(), rows.end());
            if (!rows.empty()) skids[P.col2super[rows[0]]].push_back(s);
            below[s].swap(rows);
        }
        P.srow_ptr.assign(P.nsuper + 1, 0);
        P.spanel_off.assign(P.nsuper + 1, 0);
        for (int32_t s = 0; s < P.nsuper; ++s) {
            const int64_t w = P.sfirst[s + 1] - P.sfirst[s];
            const int64_t ld = w + (int64_t)below[s].size();
            P.srow_ptr[s + 1] = P.srow_ptr[s] + ld;
            P.spanel_off[s + 1] = P.spanel_off[s] + ld * w;
        }
        P.srows.resize(P.srow_ptr[P.nsuper]);
        P.nnzL_stored = 0;
        for (int32_t s = 0; s < P.nsuper; ++s) {
            int64_t o = P.srow_ptr[s];
            const int32_t f = P.sfirst[s], l = P.sfirst[s + 1] - 1;
            for (int32_t j = f; j <= l; ++j) P.srows[o++] = j;
            for (int32_t i : below[s]) P.srows[o++] = i;
            const int64_t w = l - f + 1;
            P.nnzL_stored += w * (w + 1) / 2 + w * (int64_t)below[s].size();
        }
        P.nval = P.spanel_off[P.nsuper];
    }

    // ---- CSR entry -> panel slot
    P.kmap.assign(in.rowptr[n], -1);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t i = iperm[r];
        for (int64_t p = in.rowptr[r]; p < in.rowptr[r + 1]; ++p) {
            const int32_t j = iperm[in.col[p]];
            if (i < j) continue;
            const int32_t s = P.col2super[j];
            const int32_t* rb = P.srows.data() + P.srow_ptr[s];
            const int32_t* re = P.srows.data() + P.srow_ptr[s + 1];
            const int32_t* it = std::lower_bound(rb, re, i);
            const int64_t ld = re - rb;
            P.kmap[p] = P.spanel_off[s] + (int64_t)(j - P.sfirst[s]) * ld + (it - rb);
        }
    }

    // ---- factor flop estimate (exact structure)
    P.factor_flops = 0;
    for (int32_t j = 0; j < n; ++j) {
        const double c = P.colcount[j];
        P.factor_flops += c * c;
    }

    // ---- staircase: pivots, stable sort by (pivot, original index)
    const int32_t m = in.m;
    P.dof.assign(in.dof, in.dof + m);
    P.sign.assign(in.sign, in.sign + m);
    std::vector<int32_t> pv(m);
    for (int32_t j = 0; j < m; ++j) pv[j] = iperm[in.dof[j]];
    P.pi.resize(m);
    std::iota(P.pi.begin(), P.pi.end(), 0);
    if (opt.staircase)
        std::stable_sort(P.pi.begin(), P.pi.end(), [&](int32_t a, int32_t b) { return pv[a] < pv[b]; });
    P.piv.resize(m);
    P.sign_sorted.resize(m);
    for (int32_t k = 0; k < m; ++k) {
        P.piv[k] = pv[P.pi[k]];
        P.sign_sorted[k] = in.sign[P.pi[k]];
    }
    P.active.assign(n, 0);
    for (int32_t j = 0; j < m; ++j) P.active[pv[j]] += 1;
    for (int32_t i = 1; i < n; ++i) P.active[i] += P.active[i - 1];
    P.trsm_useful = P.syrk_useful = P.trsm_dense = 0;
    for (int32_t i = 0; i < n; ++i) {
        const double a = P.active[i], c = P.colcount[i];
        P.trsm_useful += a * (2 * c - 1);
        P.syrk_useful += a * (a + 1);
        P.trsm_dense += (double)m * (2 * c - 1);
    }
    P.syrk_dense = (double)n * (double)m * (double)(m + 1);
    // structural counts: row i of column j of X is nonzero iff i lies on the
    // elimination-tree path from j's pivot to the root, i.e. iff the pivot is
    // in the subtree of i; r(i) = pivots in that subtree (children precede
    // their parent, so one increasing pass sums the subtrees)
    {
        std::vector<double> r(n, 0.0);
        for (int32_t j = 0; j < m; ++j) r[pv[j]] += 1;
        for (int32_t i = 0; i < n; ++i)
            if (P.parent[i] >= 0) r[P.parent[i]] += r[i];
        P.trsm_reach = P.syrk_reach = 0;
        for (int32_t i = 0; i < n; ++i) {
            const double c = P.colcount[i];
            P.trsm_reach += r[i] * (2 * c - 1);
            P.syrk_reach += r[i] * (r[i] + 1);
        }
    }

    // ---- GPU blocks (Sec. 3.2, factor splitting): column ranges of at most bs
    // columns, either uniform, or following the elimination tree (the
    // non-uniform splitting of the Sec. 4.1 footnote): a block is a whole
    // subtree or the top part of one (never two unrelated subtrees), so that
    // the blocks of disjoint subtrees stay independent and a block's pruned
    // rows are not the union of unrelated row structures; a supernode wider
    // than bs is cut into bs-column panels.  Pruned rows = rows >= the block
    // end that hold a nonzero in any of the block's columns.
    const int32_t bs = std::max(16, (opt.panel_width / 16) * 16);
    P.block_width = bs;
    P.block_of_row.assign(n, -1);
    std::vector<int32_t> bstart;
    if (opt.block_split == 0) {
        for (int32_t c0 = 0; c0 < n; c0 += bs) bstart.push_back(c0);
    } else {
        // supernodal elimination tree (supernodes are in postorder); a range
        // of columns [c0, c1) is closed when every supernode in it but the
        // last has its parent in it (a subtree, or the top part of one): the
        // largest closed range of at most bs columns becomes the next block
        std::vector<int32_t> sparent(P.nsuper, -1);
        for (int32_t s = 0; s < P.nsuper; ++s) {
            const int32_t pc = P.parent[P.sfirst[s + 1] - 1];
            if (pc >= 0) sparent[s] = P.col2super[pc];
        }
        for (int32_t c0 = 0; c0 < n;) {
            bstart.push_back(c0);
            int32_t best = -1, maxpar = -1;
            for (int32_t t = P.col2super[c0]; t < P.nsuper; ++t) {
                const int32_t e = P.sfirst[t + 1];
                if (maxpar <= t) best = std::min(e, c0 + bs);   // [c0, min(e, c0 + bs)) is closed
                if (e - c0 >= bs) break;
                maxpar = std::max(maxpar, sparent[t] < 0 ? P.nsuper : sparent[t]);
            }
            c0 = best;
        }
    }
    bstart.push_back(n);
    {
        std::vector<int32_t> mark(n, -1);
        int64_t voff = 0;
        for (size_t bi = 0; bi + 1 < bstart.size(); ++bi) {
            const int32_t c0 = bstart[bi];
            const int32_t c1 = bstart[bi + 1];
            const int32_t b = (int32_t)P.blocks.size();
            std::vector<int32_t> rows;
            for (int32_t s = P.col2super[c0]; s < P.nsuper && P.sfirst[s] < c1; ++s)
                for (int64_t q = P.srow_ptr[s]; q < P.srow_ptr[s + 1]; ++q) {
                    const int32_t i = P.srows[q];
                    if (i >= c1 && mark[i] != b) { mark[i] = b; rows.push_back(i); }
                }
            std::sort(rows.begin(), rows.end());
            BlockDesc d;
            d.row0 = c0;
            d.w = c1 - c0;
            d.nbelow = (int32_t)rows.size();
            d.ld = d.w;
            d.lval_off = voff;
            while (P.brows.size() % 4) P.brows.push_back(-1);   // 16-byte aligned row lists
            d.rows_off = (int64_t)P.brows.size();
            voff += (int64_t)d.w * d.w;
            voff = (voff + 7) / 8 * 8;                  // 64-byte aligned tiles
            d.linv_off = voff;
            {
                const int64_t nrt_d = (d.w + 15) / 16, nks = (d.w + 3) / 4;
                voff += (2 * (nrt_d - 1) * nrt_d + nks) * 64;   // lower tiles only
            }
            d.aoff = voff;
            voff += (int64_t)((d.nbelow + 15) / 16) * ((d.w + 3) / 4) * 64;
            P.brows.insert(P.brows.end(), rows.begin(), rows.end());
            for (int32_t i = c0; i < c1; ++i) P.block_of_row[i] = b;
            P.blocks.push_back(d);
        }
        P.bval = voff;
    }

    // ---- blocks each 64-column tile of X visits.  Column c of X = L^{-1} P B^T
    // is nonzero only on the elimination-tree path from its pivot to the root
    // (the reach of one right-hand-side entry); a factor block none of whose
    // rows lies on the path of any of the tile's columns holds zero rows of
    // the tile and contributes nothing, so the sweep skips it.  Without the
    // reach the sweep runs from the first pivot's block to the last block
    // (the staircase alone), without the staircase over every block.
    {
        const int32_t nb = (int32_t)P.blocks.size();
        const int32_t ntile = (m + 63) / 64;
        std::vector<int32_t> stamp(n, -1), bstamp(nb, -1), bpos(nb, 0);
        P.visit_ptr.assign(1, 0);
        P.visit.clear();
        P.visit_rows.clear();
        std::vector<int32_t> rr;
        P.visits_stair = 0;
        P.mask_words = (n + 16 * 64 - 1) / (16 * 64);
        P.step_mask.assign((size_t)ntile * P.mask_words, 0);
        for (int32_t t = 0; t < ntile; ++t) {
            const int32_t c0 = 64 * t, c1 = std::min(m, c0 + 64);
            const int32_t first = opt.staircase ? P.block_of_row[P.piv[c0]] : 0;
            uint64_t* mask = P.step_mask.data() + (size_t)t * P.mask_words;
            P.visits_stair += nb - first;
            if (!opt.staircase || !opt.reach) {
                for (int32_t b = first; b < nb; ++b) {
                    P.visit.push_back(b);
                    P.visit_rows.push_back(P.blocks[b].w >= 64 ? ~0ull : (1ull << P.blocks[b].w) - 1);
                }
                for (int32_t q = (opt.staircase ? P.piv[c0] : 0) / 16; q < (n + 15) / 16; ++q)
                    mask[q >> 6] |= 1ull << (q & 63);
            } else {
                std::vector<int32_t> bl;
                rr.clear();
                for (int32_t c = c0; c < c1; ++c)
                    for (int32_t r = P.piv[c]; r >= 0 && stamp[r] != t; r = P.parent[r]) {
                        stamp[r] = t;
                        rr.push_back(r);
                        mask[r >> 10] |= 1ull << ((r >> 4) & 63);
                        const int32_t b = P.block_of_row[r];
                        if (bstamp[b] != t) { bstamp[b] = t; bl.push_back(b); }
                    }
                std::sort(bl.begin(), bl.end());
                const size_t v0 = P.visit.size();
                for (size_t q = 0; q < bl.size(); ++q) bpos[bl[q]] = (int32_t)q;
                P.visit.insert(P.visit.end(), bl.begin(), bl.end());
                P.visit_rows.resize(P.visit.size(), 0);
                for (int32_t r : rr) {
                    const int32_t b = P.block_of_row[r];
                    P.visit_rows[v0 + bpos[b]] |= 1ull << (r - P.blocks[b].row0);
                }
            }
            P.visit_ptr.push_back((int64_t)P.visit.size());
        }
    }
    code = 0;
    return "";
}

// ---------------------------------------------------------------------------
// numeric supernodal Cholesky: for each supernode in order, factor its panel
// (the (w + r) x w block column: Cholesky of the w x w diagonal block and the
// triangular solve of the r rows below, left-looking over column blocks of
// kPanelBlock, the update of each block a product with the columns before it),
// then subtract its outer-product contribution from every later supernode its
// rows touch (right-looking: one product per target supernode into a dense
// buffer, scattered into the target's panel).
// ---------------------------------------------------------------------------
namespace {
constexpr int32_t kPanelBlock = 32;
constexpr int64_t kUpdateBlock = 64;
}

int64_t factor_numeric(const SubPlan& P, const double* kvals, double* vals) {
    std::memset(vals, 0, sizeof(double) * (size_t)P.nval);
    for (size_t e = 0; e < P.kmap.size(); ++e)
        if (P.kmap[e] >= 0) vals[P.kmap[e]] += kvals[e];
    std::vector<int32_t> pos(P.n, -1);
    std::vector<double> tmp;
    for (int32_t s = 0; s < P.nsuper; ++s) {
        const int32_t f = P.sfirst[s];
        const int32_t w = P.sfirst[s + 1] - f;
        const int64_t ld = P.srow_ptr[s + 1] - P.srow_ptr[s];
        double* A = vals + P.spanel_off[s];
        const int32_t* rows = P.srows.data() + P.srow_ptr[s];
        for (int32_t j0 = 0; j0 < w; j0 += kPanelBlock) {
            const int32_t j1 = std::min(w, j0 + kPanelBlock);
            // columns [j0, j1) minus the contributions of columns [0, j0)
            // (rows j0.. of both; the entries above the diagonal that this
            // also updates are never read)
            gemm_nt(ld - j0, j1 - j0, j0, -1.0, A + j0, ld, A + j0, ld, A + j0 + (size_t)j0 * ld, ld);
            for (int32_t c = j0; c < j1; ++c) {
                double* colc = A + (size_t)c * ld;
                for (int32_t k = j0; k < c; ++k) {
                    const double* colk = A + (size_t)k * ld;
                    const double lck = colk[c];
                    if (lck == 0.0) continue;
                    for (int64_t i = c; i < ld; ++i) colc[i] -= colk[i] * lck;
                }
                const double d = colc[c];
                if (!(d > 0.0)) return f + c;
                const double sd = std::sqrt(d);
                colc[c] = sd;
                const double inv = 1.0 / sd;
                for (int64_t i = c + 1; i < ld; ++i) colc[i] *= inv;
            }
        }
        // contributions to later supernodes
        int64_t q = w;
        while (q < ld) {
            const int32_t t = P.col2super[rows[q]];
            const int32_t tf = P.sfirst[t];
            const int32_t tl = P.sfirst[t + 1] - 1;
            int64_t q1 = q;
            while (q1 < ld && rows[q1] <= tl) ++q1;
            const int64_t ldt = P.srow_ptr[t + 1] - P.srow_ptr[t];
            const int32_t* trows = P.srows.data() + P.srow_ptr[t];
            for (int64_t k = 0; k < ldt; ++k) pos[trows[k]] = (int32_t)k;
            double* T = vals + P.spanel_off[t];
            const int64_t nr = ld - q, nb = q1 - q;
            // tmp = L[q:ld, :] L[q:q1, :]^T (nr x nb), on and below the
            // diagonal of its top nb x nb block: column block [b0, b1) from
            // row b0 down
            tmp.resize((size_t)(nr * nb));
            for (int64_t b0 = 0; b0 < nb; b0 += kUpdateBlock) {
                const int64_t b1 = std::min(nb, b0 + kUpdateBlock);
                for (int64_t b = b0; b < b1; ++b) std::fill(tmp.begin() + b * nr + b0, tmp.begin() + (b + 1) * nr, 0.0);
                gemm_nt(nr - b0, b1 - b0, w, 1.0, A + q + b0, ld, A + q + b0, ld, tmp.data() + b0 * nr + b0, nr);
            }
            for (int64_t b = 0; b < nb; ++b) {
                double* tcol = T + (size_t)(rows[q + b] - tf) * ldt;
                const double* src = tmp.data() + b * nr;
                for (int64_t a = b; a < nr; ++a) tcol[pos[rows[q + a]]] -= src[a];
            }
            q = q1;
        }
    }
    return -1;
}

std::vector<int32_t> merge_pairs(const SubPlan& P) {
    const int32_t nb = (int32_t)P.blocks.size();
    std::vector<int32_t> flag(nb, 0);
    for (int32_t b = 0; b + 1 < nb; ++b) {
        if (b > 0 && flag[b - 1]) continue;           // b is the second block of a pair
        const BlockDesc& x = P.blocks[b];
        const BlockDesc& y = P.blocks[b + 1];
        if (y.w % 16 != 0 || x.nbelow != y.w + y.nbelow) continue;
        bool same = true;
        for (int32_t q = 0; q < y.w && same; ++q) same = P.brows[x.rows_off + q] == y.row0 + q;
        for (int32_t q = 0; q < y.nbelow && same; ++q) same = P.brows[x.rows_off + y.w + q] == P.brows[y.rows_off + q];
        if (same) flag[b] = 1;
    }
    return flag;
}

void repack_blocks(const SubPlan& P, const double* vals, double* bvals) {
    std::memset(bvals, 0, sizeof(double) * (size_t)P.bval);
    std::vector<int32_t> pos(P.n, -1);
    for (const BlockDesc& b : P.blocks) {
        const int32_t c0 = b.row0, c1 = b.row0 + b.w;
        const int64_t nks = (b.w + 3) / 4;
        for (int32_t q = 0; q < b.nbelow; ++q) pos[P.brows[b.rows_off + q]] = b.w + q;
        for (int32_t i = c0; i < c1; ++i) pos[i] = i - c0;
        double* diag = bvals + b.lval_off;
        double* at = bvals + b.aoff;
        for (int32_t s = P.col2super[c0]; s < P.nsuper && P.sfirst[s] < c1; ++s) {
            const int32_t f = P.sfirst[s];
            const int64_t ld = P.srow_ptr[s + 1] - P.srow_ptr[s];
            const int32_t* rows = P.srows.data() + P.srow_ptr[s];
            const double* A = vals + P.spanel_off[s];
            const int32_t j0 = std::max(c0, f), j1 = std::min(c1, P.sfirst[s + 1]);
            for (int32_t j = j0; j < j1; ++j) {
                const int32_t cj = j - f, k = j - c0;
                for (int64_t q = cj; q < ld; ++q) {
                    const int32_t p = pos[rows[q]];
                    const double v = A[(size_t)cj * ld + q];
                    if (p < b.w) {
                        diag[(size_t)k * b.w + p] = v;
                    } else {
                        const int32_t r = p - b.w;
                        at[((r / 16) * nks + k / 4) * 64 + (r % 16) + 16 * (k % 4)] = v;
                    }
                }
            }
        }
        // inverse of the diagonal triangle, column by column (forward
        // substitution on the unit vectors, accumulated in long double)
        const int32_t w = b.w;
        double* li = bvals + b.linv_off;
        std::vector<long double> z(w);
        for (int32_t c = 0; c < w; ++c) {
            for (int32_t i = c; i < w; ++i) {
                long double acc = (i == c) ? 1.0L : 0.0L;
                for (int32_t k = c; k < i; ++k) acc -= (long double)diag[(size_t)k * w + i] * z[k];
                z[i] = acc / (long double)diag[(size_t)i * w + i];
                const int64_t rt = i / 16;
                li[(2 * rt * (rt + 1) + c / 4) * 64 + (i % 16) + 16 * (c % 4)] = (double)z[i];
            }
        }
    }
}

}  // namespace scasm
