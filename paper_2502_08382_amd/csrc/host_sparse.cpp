// Nested dissection, supernodal symbolic analysis and numeric multifrontal
// Cholesky for the regularised subdomain stiffness K_reg = L L^T.
#include "host_sparse.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace fetif {

// ---------------------------------------------------------------- ordering

namespace {

struct NodeGraph {
    int32_t n = 0;
    std::vector<int32_t> ptr, adj;
};

NodeGraph node_graph(const Pattern& A, int dpn)
{
    NodeGraph g;
    g.n = A.n / dpn;
    std::vector<std::vector<int32_t>> nb(g.n);
    for (int32_t r = 0; r < A.n; ++r) {
        int32_t a = r / dpn;
        for (int32_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
            int32_t b = A.idx[p] / dpn;
            if (b != a) nb[a].push_back(b);
        }
    }
    g.ptr.assign(g.n + 1, 0);
    for (int32_t a = 0; a < g.n; ++a) {
        auto& v = nb[a];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        g.ptr[a + 1] = g.ptr[a] + (int32_t)v.size();
    }
    g.adj.resize(g.ptr[g.n]);
    for (int32_t a = 0; a < g.n; ++a) std::copy(nb[a].begin(), nb[a].end(), g.adj.begin() + g.ptr[a]);
    return g;
}

struct NDState {
    const NodeGraph* g;
    const double* xyz;
    int dim;
    int leaf;
    std::vector<int32_t> side;  // scratch label per node
    std::vector<int32_t> order;
};

// breadth-first level structure restricted to the nodes labelled `lab`
static std::vector<int32_t> bfs_levels(NDState& st, const std::vector<int32_t>& nodes, int32_t root,
                                       int32_t lab, std::vector<int32_t>& level)
{
    std::vector<int32_t> q;
    q.reserve(nodes.size());
    for (int32_t v : nodes) level[v] = -1;
    level[root] = 0;
    q.push_back(root);
    for (size_t h = 0; h < q.size(); ++h) {
        int32_t v = q[h];
        for (int32_t p = st.g->ptr[v]; p < st.g->ptr[v + 1]; ++p) {
            int32_t w = st.g->adj[p];
            if (st.side[w] == lab && level[w] < 0) {
                level[w] = level[v] + 1;
                q.push_back(w);
            }
        }
    }
    return q;
}

static void nd_rec(NDState& st, std::vector<int32_t> nodes, int depth)
{
    const size_t N = nodes.size();
    if (N == 0) return;
    if ((int)N <= st.leaf || depth > 64) {
        std::sort(nodes.begin(), nodes.end());
        st.order.insert(st.order.end(), nodes.begin(), nodes.end());
        return;
    }
    const int32_t LAB = 1, LEFT = 2, RIGHT = 3, SEP = 4;
    for (int32_t v : nodes) st.side[v] = LAB;
    bool split = false;
    if (st.xyz) {
        int axis = 0;
        double best = -1.0;
        for (int d = 0; d < st.dim; ++d) {
            double lo = 1e300, hi = -1e300;
            for (int32_t v : nodes) {
                double x = st.xyz[(size_t)v * st.dim + d];
                lo = std::min(lo, x);
                hi = std::max(hi, x);
            }
            if (hi - lo > best) { best = hi - lo; axis = d; }
        }
        if (best > 0.0) {
            std::vector<double> xs(N);
            for (size_t k = 0; k < N; ++k) xs[k] = st.xyz[(size_t)nodes[k] * st.dim + axis];
            std::vector<double> u(xs);
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            // the plane holding the median node
            std::vector<double> srt(xs);
            std::nth_element(srt.begin(), srt.begin() + N / 2, srt.end());
            double v = srt[N / 2];
            if (u.size() >= 3) {
                if (v == u.front()) v = u[1];
                if (v == u.back()) v = u[u.size() - 2];
                for (size_t k = 0; k < N; ++k)
                    st.side[nodes[k]] = xs[k] < v ? LEFT : (xs[k] > v ? RIGHT : SEP);
            } else {
                for (size_t k = 0; k < N; ++k) st.side[nodes[k]] = xs[k] == u.front() ? LEFT : RIGHT;
            }
            split = true;
        }
    }
    if (!split) {
        // graph fallback: middle level of a BFS from a pseudo-peripheral node
        std::vector<int32_t> level(st.side.size(), -1);
        int32_t root = nodes[0];
        int32_t last_depth = -1;
        std::vector<int32_t> q;
        for (int it = 0; it < 4; ++it) {
            q = bfs_levels(st, nodes, root, LAB, level);
            int32_t far = q.back();
            if (level[far] <= last_depth) break;
            last_depth = level[far];
            root = far;
        }
        q = bfs_levels(st, nodes, root, LAB, level);
        if (q.size() < N) {
            // disconnected: the component of root against the rest, no separator
            for (int32_t v : nodes) st.side[v] = level[v] >= 0 ? LEFT : RIGHT;
        } else {
            int32_t maxl = level[q.back()];
            if (maxl < 2) {
                std::sort(nodes.begin(), nodes.end());
                st.order.insert(st.order.end(), nodes.begin(), nodes.end());
                return;
            }
            // level at which about half of the nodes lie below
            std::vector<int32_t> cnt(maxl + 1, 0);
            for (int32_t v : nodes) cnt[level[v]]++;
            int32_t acc = 0, mid = 1;
            for (int32_t l = 0; l <= maxl; ++l) {
                acc += cnt[l];
                if (acc * 2 >= (int32_t)N) { mid = std::max(1, std::min(l, maxl - 1)); break; }
            }
            for (int32_t v : nodes) st.side[v] = level[v] < mid ? LEFT : (level[v] > mid ? RIGHT : SEP);
        }
    }
    // complete to a vertex separator: right endpoints of left-right edges
    for (int32_t v : nodes) {
        if (st.side[v] != LEFT) continue;
        for (int32_t p = st.g->ptr[v]; p < st.g->ptr[v + 1]; ++p) {
            int32_t w = st.g->adj[p];
            if (st.side[w] == RIGHT) st.side[w] = SEP;
        }
    }
    std::vector<int32_t> L, R, S;
    for (int32_t v : nodes) {
        if (st.side[v] == LEFT) L.push_back(v);
        else if (st.side[v] == RIGHT) R.push_back(v);
        else S.push_back(v);
    }
    for (int32_t v : nodes) st.side[v] = 0;
    if (L.empty() || R.empty()) {
        if (L.size() + S.size() == N || R.size() + S.size() == N) {
            // no progress possible on this set
            std::sort(nodes.begin(), nodes.end());
            st.order.insert(st.order.end(), nodes.begin(), nodes.end());
            return;
        }
    }
    nd_rec(st, std::move(L), depth + 1);
    nd_rec(st, std::move(R), depth + 1);
    std::sort(S.begin(), S.end());
    st.order.insert(st.order.end(), S.begin(), S.end());
}

}  // namespace

std::vector<int32_t> nested_dissection(const Pattern& A, int dpn, const double* coords, int dim,
                                       int leaf_nodes, const std::vector<char>* last)
{
    NodeGraph g = node_graph(A, dpn);
    NDState st;
    st.g = &g;
    st.xyz = coords;
    st.dim = dim;
    st.leaf = std::max(1, leaf_nodes);
    st.side.assign(g.n, 0);
    std::vector<int32_t> all, tail;
    all.reserve(g.n);
    for (int32_t v = 0; v < g.n; ++v) {
        if (last && (*last)[v]) tail.push_back(v);
        else all.push_back(v);
    }
    nd_rec(st, std::move(all), 0);
    st.order.insert(st.order.end(), tail.begin(), tail.end());
    std::vector<int32_t> perm((size_t)A.n);
    for (int32_t k = 0; k < g.n; ++k)
        for (int c = 0; c < dpn; ++c) perm[(size_t)k * dpn + c] = st.order[k] * dpn + c;
    return perm;
}

// ---------------------------------------------------------------- symbolic

namespace {

void permuted_lower(const Pattern& A, const std::vector<int32_t>& perm, const std::vector<int32_t>& pinv,
                    std::vector<int32_t>& cptr, std::vector<int32_t>& crow, std::vector<int32_t>& csrc)
{
    const int32_t n = A.n;
    cptr.assign(n + 1, 0);
    for (int32_t j = 0; j < n; ++j) {
        int32_t o = perm[j];
        for (int32_t p = A.ptr[o]; p < A.ptr[o + 1]; ++p)
            if (pinv[A.idx[p]] >= j) cptr[j + 1]++;
    }
    for (int32_t j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
    crow.resize(cptr[n]);
    csrc.resize(cptr[n]);
    std::vector<std::pair<int32_t, int32_t>> tmp;
    for (int32_t j = 0; j < n; ++j) {
        tmp.clear();
        int32_t o = perm[j];
        for (int32_t p = A.ptr[o]; p < A.ptr[o + 1]; ++p) {
            int32_t i = pinv[A.idx[p]];
            if (i >= j) tmp.emplace_back(i, p);
        }
        std::sort(tmp.begin(), tmp.end());
        for (size_t k = 0; k < tmp.size(); ++k) {
            crow[cptr[j] + k] = tmp[k].first;
            csrc[cptr[j] + k] = tmp[k].second;
        }
    }
}

// etree from the lower triangle stored by columns: row i's upper entries
// are the (i, j) with j < i, i.e. column j lists row i.
std::vector<int32_t> etree_lower(int32_t n, const std::vector<int32_t>& cptr, const std::vector<int32_t>& crow)
{
    // transpose to get, for each row i, the columns j < i
    std::vector<int32_t> rptr(n + 1, 0), rcol(cptr[n]);
    for (int32_t j = 0; j < n; ++j)
        for (int32_t p = cptr[j]; p < cptr[j + 1]; ++p) rptr[crow[p] + 1]++;
    for (int32_t i = 0; i < n; ++i) rptr[i + 1] += rptr[i];
    std::vector<int32_t> nxt(rptr.begin(), rptr.end() - 1);
    for (int32_t j = 0; j < n; ++j)
        for (int32_t p = cptr[j]; p < cptr[j + 1]; ++p) rcol[nxt[crow[p]]++] = j;
    std::vector<int32_t> parent(n, -1), anc(n, -1);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t p = rptr[i]; p < rptr[i + 1]; ++p) {
            int32_t j = rcol[p];
            while (j != -1 && j < i) {
                int32_t nx = anc[j];
                anc[j] = i;
                if (nx == -1) parent[j] = i;
                j = nx;
            }
        }
    }
    return parent;
}

std::vector<int32_t> postorder(const std::vector<int32_t>& parent)
{
    const int32_t n = (int32_t)parent.size();
    std::vector<int32_t> head(n, -1), next(n, -1), post;
    post.reserve(n);
    for (int32_t j = n - 1; j >= 0; --j) {
        if (parent[j] >= 0) {
            next[j] = head[parent[j]];
            head[parent[j]] = j;
        }
    }
    std::vector<int32_t> stack;
    for (int32_t r = 0; r < n; ++r) {
        if (parent[r] != -1) continue;
        stack.push_back(r);
        while (!stack.empty()) {
            int32_t v = stack.back();
            int32_t c = head[v];
            if (c == -1) {
                post.push_back(v);
                stack.pop_back();
            } else {
                head[v] = next[c];
                stack.push_back(c);
            }
        }
    }
    return post;
}

}  // namespace

bool symbolic_analysis(const Pattern& A, int dpn, const double* coords, int dim,
                       const SymbolicOptions& opt, Symbolic& S, std::string& err)
{
    const int32_t n = A.n;
    if (n <= 0 || dpn <= 0 || n % dpn != 0 || (int32_t)A.ptr.size() != n + 1) {
        err = "invalid pattern or dofs-per-node";
        return false;
    }
    for (int32_t r = 0; r < n; ++r)
        for (int32_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p)
            if (A.idx[p] < 0 || A.idx[p] >= n) {
                err = "column index out of range";
                return false;
            }
    if (opt.last_nodes && (int64_t)opt.last_nodes->size() != n / dpn) {
        err = "node flag count does not match the pattern";
        return false;
    }
    std::vector<int32_t> perm = nested_dissection(A, dpn, coords, dim, opt.leaf_nodes, opt.last_nodes);
    std::vector<int32_t> pinv(n);
    for (int32_t k = 0; k < n; ++k) pinv[perm[k]] = k;
    std::vector<int32_t> cptr, crow, csrc;
    permuted_lower(A, perm, pinv, cptr, crow, csrc);
    std::vector<int32_t> parent = etree_lower(n, cptr, crow);
    // relabel in postorder
    std::vector<int32_t> post = postorder(parent);
    std::vector<int32_t> perm2(n), ipost(n);
    for (int32_t k = 0; k < n; ++k) {
        perm2[k] = perm[post[k]];
        ipost[post[k]] = k;
    }
    perm.swap(perm2);
    for (int32_t k = 0; k < n; ++k) pinv[perm[k]] = k;
    permuted_lower(A, perm, pinv, cptr, crow, csrc);
    {
        std::vector<int32_t> p2(n);
        for (int32_t k = 0; k < n; ++k) p2[k] = parent[post[k]] < 0 ? -1 : ipost[parent[post[k]]];
        parent.swap(p2);
    }
    // column structures below the diagonal, children before parents
    std::vector<std::vector<int32_t>> st(n);
    std::vector<int32_t> nchild(n, 0);
    std::vector<std::vector<int32_t>> children(n);
    for (int32_t j = 0; j < n; ++j)
        if (parent[j] >= 0) {
            nchild[parent[j]]++;
            children[parent[j]].push_back(j);
        }
    std::vector<int32_t> mark(n, -1);
    for (int32_t j = 0; j < n; ++j) {
        auto& s = st[j];
        mark[j] = j;
        for (int32_t p = cptr[j]; p < cptr[j + 1]; ++p) {
            int32_t i = crow[p];
            if (mark[i] != j) { mark[i] = j; s.push_back(i); }
        }
        for (int32_t c : children[j]) {
            for (int32_t i : st[c]) {
                if (mark[i] != j) { mark[i] = j; s.push_back(i); }
            }
        }
        std::sort(s.begin(), s.end());
        // a child's structure is not needed once its parent is built, except
        // for supernode rows; keep only those of possible supernode tops
    }
    std::vector<int32_t> cc(n);
    for (int32_t j = 0; j < n; ++j) cc[j] = (int32_t)st[j].size() + 1;
    // fundamental supernodes
    std::vector<int32_t> sfirst;
    for (int32_t j = 0; j < n; ++j) {
        bool cont = j > 0 && parent[j - 1] == j && nchild[j] == 1 && cc[j - 1] == cc[j] + 1;
        if (!cont) sfirst.push_back(j);
    }
    int32_t ns0 = (int32_t)sfirst.size();
    std::vector<int32_t> sf(sfirst), sl(ns0);
    for (int32_t s = 0; s < ns0; ++s) sl[s] = (s + 1 < ns0 ? sfirst[s + 1] : n);  // exclusive end
    std::vector<int32_t> c2s(n);
    for (int32_t s = 0; s < ns0; ++s)
        for (int32_t j = sf[s]; j < sl[s]; ++j) c2s[j] = s;
    // relaxed amalgamation of a supernode with the child that immediately
    // precedes it; c2s maps a column to its current representative
    std::vector<int32_t> alive(ns0, 1), first(sf), last(sl);
    std::vector<double> zeros(ns0, 0.0);  // explicit zeros inside a supernode
    auto nrows_of = [&](int32_t s) { return (int32_t)st[last[s] - 1].size(); };
    auto rep_parent = [&](int32_t s) {
        int32_t pj = parent[last[s] - 1];
        return pj < 0 ? -1 : c2s[pj];
    };
    for (int32_t p = 0; p < ns0; ++p) {
        for (;;) {
            if (first[p] == 0) break;
            int32_t c = c2s[first[p] - 1];
            if (!alive[c] || rep_parent(c) != p) break;
            int32_t ncol = last[p] - first[c];
            int32_t nr = nrows_of(p);
            double z = zeros[p], tot = 0.0;
            for (int32_t j = first[c]; j < last[c]; ++j) z += (double)((last[p] - j) + nr - cc[j]);
            for (int32_t j = first[c]; j < last[p]; ++j) tot += (double)((last[p] - j) + nr);
            double frac = z / std::max(1.0, tot);
            bool ok = (ncol <= opt.relax_cols[0]) ||
                      (ncol <= opt.relax_cols[1] && frac <= opt.relax_zeros[0]) ||
                      (ncol <= opt.relax_cols[2] && frac <= opt.relax_zeros[1]) ||
                      (ncol <= opt.relax_cols[3] && frac <= opt.relax_zeros[2]);
            if (!ok) break;
            alive[c] = 0;
            for (int32_t j = first[c]; j < last[c]; ++j) c2s[j] = p;
            first[p] = first[c];
            zeros[p] = z;
        }
    }
    // final supernodes in column order
    S = Symbolic();
    S.n = n;
    S.perm = perm;
    S.pinv = pinv;
    std::vector<int32_t> newid(ns0, -1);
    for (int32_t s = 0; s < ns0; ++s) {
        if (!alive[s]) continue;
        newid[s] = (int32_t)S.sn.size();
        Supernode x;
        x.first = first[s];
        x.ncols = last[s] - first[s];
        x.nrows = nrows_of(s);
        S.sn.push_back(x);
    }
    // supernodes are generated in increasing first column since alive
    // representatives keep the column order of their top part
    std::sort(S.sn.begin(), S.sn.end(), [](const Supernode& a, const Supernode& b) { return a.first < b.first; });
    const int32_t ns = (int32_t)S.sn.size();
    S.col2sn.assign(n, -1);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t j = S.sn[s].first; j < S.sn[s].first + S.sn[s].ncols; ++j) S.col2sn[j] = s;
    int64_t roff = 0, voff = 0;
    S.flops_factor = 0.0;
    for (int32_t s = 0; s < ns; ++s) {
        Supernode& x = S.sn[s];
        int32_t lastc = x.first + x.ncols - 1;
        const auto& rows = st[lastc];
        x.row_off = roff;
        x.val_off = voff;
        S.rows.insert(S.rows.end(), rows.begin(), rows.end());
        roff += (int64_t)rows.size();
        voff += (int64_t)(x.ncols + x.nrows) * x.ncols;
        x.parent = parent[lastc] < 0 ? -1 : S.col2sn[parent[lastc]];
        double d = x.ncols + x.nrows;
        for (int32_t k = 0; k < x.ncols; ++k) {
            double h = d - k;
            S.flops_factor += h * h;
        }
    }
    S.nvals = voff;
    // heights
    int32_t maxl = 0;
    for (int32_t s = 0; s < ns; ++s) {
        Supernode& x = S.sn[s];
        if (x.parent >= 0) S.sn[x.parent].level = std::max(S.sn[x.parent].level, x.level + 1);
        maxl = std::max(maxl, x.level);
    }
    S.nlevels = maxl + 1;
    S.acol_ptr.swap(cptr);
    S.acol_row.swap(crow);
    S.acol_src.swap(csrc);
    return true;
}

// ---------------------------------------------------------------- numeric

namespace {

// out[i] -= sum_{t < nk} l[t] * col[t][i] for i in [i0, i1); nk <= 16,
// the sum in t order for each i.  The same code is compiled twice: for the
// baseline x86-64 target and for AVX2 + FMA, chosen once at run time.
#define FETIF_AXPY_BLOCK_BODY                                                                                      \
    switch (nk) {                                                                                                  \
    case 16:                                                                                                       \
        for (int32_t i = i0; i < i1; ++i)                                                                          \
            out[i] -= ((l[0] * col[0][i] + l[1] * col[1][i] + l[2] * col[2][i] + l[3] * col[3][i]) +              \
                       (l[4] * col[4][i] + l[5] * col[5][i] + l[6] * col[6][i] + l[7] * col[7][i])) +             \
                      ((l[8] * col[8][i] + l[9] * col[9][i] + l[10] * col[10][i] + l[11] * col[11][i]) +          \
                       (l[12] * col[12][i] + l[13] * col[13][i] + l[14] * col[14][i] + l[15] * col[15][i]));      \
        return;                                                                                                    \
    case 8:                                                                                                        \
        for (int32_t i = i0; i < i1; ++i)                                                                          \
            out[i] -= (l[0] * col[0][i] + l[1] * col[1][i] + l[2] * col[2][i] + l[3] * col[3][i]) +               \
                      (l[4] * col[4][i] + l[5] * col[5][i] + l[6] * col[6][i] + l[7] * col[7][i]);                \
        return;                                                                                                    \
    default:                                                                                                       \
        for (int32_t i = i0; i < i1; ++i) {                                                                        \
            double a = 0.0;                                                                                        \
            for (int32_t t = 0; t < nk; ++t) a += l[t] * col[t][i];                                                \
            out[i] -= a;                                                                                           \
        }                                                                                                          \
    }

void axpy_block_base(double* out, int32_t i0, int32_t i1, const double* l, const double* const* col, int32_t nk)
{
    FETIF_AXPY_BLOCK_BODY
}

__attribute__((target("avx2,fma"))) void axpy_block_avx2(double* out, int32_t i0, int32_t i1, const double* l,
                                                          const double* const* col, int32_t nk)
{
    FETIF_AXPY_BLOCK_BODY
}
#undef FETIF_AXPY_BLOCK_BODY

using AxpyFn = void (*)(double*, int32_t, int32_t, const double*, const double* const*, int32_t);
const AxpyFn axpy_block = (__builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma")) ? axpy_block_avx2
                                                                                          : axpy_block_base;

// Columns j in [j0, j1) of the column-major front F (leading dimension d)
// take the rank-(k1 - k0) update of factored columns [k0, k1): F[i][j] -=
// sum_k F[i][k] F[j][k] for rows i >= j.
void rank_update(double* F, int32_t d, int32_t k0, int32_t k1, int32_t j0, int32_t j1, int32_t)
{
    for (int32_t j = j0; j < j1; ++j) {
        double l[16];
        const double* lk[16];
        int32_t nk = 0;
        for (int32_t k = k0; k < k1; ++k) {
            const double v = F[(size_t)k * d + j];
            if (v == 0.0) continue;
            l[nk] = v;
            lk[nk++] = F + (size_t)k * d;
        }
        if (nk) axpy_block(F + (size_t)j * d, j, d, l, lk, nk);
    }
}

}  // namespace

int32_t numeric_cholesky(const Symbolic& S, const double* vals, double* panels)
{
    const int32_t n = S.n;
    const int32_t ns = (int32_t)S.sn.size();
    std::vector<int32_t> pos(n, -1);
    std::vector<std::vector<double>> upd(ns);
    std::vector<std::vector<int32_t>> children(ns);
    for (int32_t s = 0; s < ns; ++s)
        if (S.sn[s].parent >= 0) children[S.sn[s].parent].push_back(s);
    std::vector<double> F;
    for (int32_t s = 0; s < ns; ++s) {
        const Supernode& x = S.sn[s];
        const int32_t nc = x.ncols, d = x.ncols + x.nrows;
        const int32_t* rows = S.rows.data() + x.row_off;
        for (int32_t k = 0; k < nc; ++k) pos[x.first + k] = k;
        for (int32_t k = 0; k < x.nrows; ++k) pos[rows[k]] = nc + k;
        F.assign((size_t)d * d, 0.0);
        auto at = [&](int32_t i, int32_t j) -> double& { return F[(size_t)j * d + i]; };
        for (int32_t k = 0; k < nc; ++k) {
            int32_t j = x.first + k;
            for (int32_t p = S.acol_ptr[j]; p < S.acol_ptr[j + 1]; ++p) at(pos[S.acol_row[p]], k) += vals[S.acol_src[p]];
        }
        for (int32_t c : children[s]) {
            const Supernode& y = S.sn[c];
            const int32_t* cr = S.rows.data() + y.row_off;
            const int32_t m = y.nrows;
            const std::vector<double>& U = upd[c];
            for (int32_t b = 0; b < m; ++b) {
                int32_t jb = pos[cr[b]];
                double* col = &F[(size_t)jb * d];
                const double* ucol = &U[(size_t)b * m];
                for (int32_t a = b; a < m; ++a) col[pos[cr[a]]] += ucol[a];
            }
            std::vector<double>().swap(upd[c]);
        }
        // partial dense Cholesky of the front, the nc pivot columns, by
        // blocks of kBlk columns: a block is factored column by column, then
        // the front's later pivot columns take its kBlk columns at once (one
        // pass over each target column per block instead of one per column)
        constexpr int32_t kBlk = 16;
        for (int32_t k0 = 0; k0 < nc; k0 += kBlk) {
            const int32_t k1 = std::min(nc, k0 + kBlk);
            for (int32_t k = k0; k < k1; ++k) {
                double* ck = &F[(size_t)k * d];
                double piv = ck[k];
                if (!(piv > 0.0) || !std::isfinite(piv)) return x.first + k;
                double r = std::sqrt(piv);
                ck[k] = r;
                double inv = 1.0 / r;
                for (int32_t i = k + 1; i < d; ++i) ck[i] *= inv;
                for (int32_t j = k + 1; j < k1; ++j) {
                    double l = ck[j];
                    if (l == 0.0) continue;
                    double* cj = &F[(size_t)j * d];
                    for (int32_t i = j; i < d; ++i) cj[i] -= ck[i] * l;
                }
            }
            rank_update(F.data(), d, k0, k1, k1, nc, k1);
        }
        // update matrix for the parent: F22 - L21 L21^T (lower part), by
        // blocks of kBlk columns of L21
        const int32_t m = x.nrows;
        if (m > 0 && x.parent >= 0) {
            std::vector<double>& U = upd[s];
            U.assign((size_t)m * m, 0.0);
            for (int32_t b = 0; b < m; ++b) {
                double* ucol = &U[(size_t)b * m];
                const double* fcol = &F[(size_t)(nc + b) * d + nc];
                for (int32_t a = b; a < m; ++a) ucol[a] = fcol[a];
            }
            for (int32_t k0 = 0; k0 < nc; k0 += kBlk) {
                const int32_t k1 = std::min(nc, k0 + kBlk);
                // U[a][b] -= sum_k L21[a][k] L21[b][k], L21 column k at F + k d + nc
                for (int32_t b = 0; b < m; ++b) {
                    double l[kBlk] = {0};
                    const double* lk[kBlk] = {nullptr};
                    int32_t nk = 0;
                    for (int32_t k = k0; k < k1; ++k) {
                        const double v = F[(size_t)k * d + nc + b];
                        if (v == 0.0) continue;
                        l[nk] = v;
                        lk[nk++] = &F[(size_t)k * d + nc];
                    }
                    if (!nk) continue;
                    double* ucol = &U[(size_t)b * m];
                    axpy_block(ucol, b, m, l, lk, nk);
                }
            }
        }
        std::memcpy(panels + x.val_off, F.data(), sizeof(double) * (size_t)d * nc);
        for (int32_t k = 0; k < nc; ++k) pos[x.first + k] = -1;
        for (int32_t k = 0; k < x.nrows; ++k) pos[rows[k]] = -1;
    }
    return -1;
}

}  // namespace fetif
