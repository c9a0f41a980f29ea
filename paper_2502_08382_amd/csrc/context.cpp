// The fetiF context: preparation (ordering, symbolic analysis, schedules,
// device structures), per-step factorisation + upload, assembly and
// application (paper Alg. 2 and Sec. IV-B).
#include <sched.h>

#include "context.hpp"

thread_local std::string fetif::g_create_error;

namespace {

bool plan_subdomain(const fetiF_subdomain& in, const fetiF_options& opt, int64_t n_lambda, SubPlan& P)
{
    Pattern A;
    if (!pattern_from_sub(in, A, P.err)) return false;
    P.n = in.n;
    P.m = in.m;
    P.dpn = in.dofs_per_node;
    P.nnzA = A.ptr[in.n];
    if (in.m <= 0 || !in.b_dof || !in.b_sign || !in.dual_map) {
        // a subdomain without multipliers is not coupled to the problem
        P.err = "every subdomain needs m >= 1 rows of B~ (b_dof, b_sign, dual_map)";
        return false;
    }
    P.b_dof.assign(in.b_dof, in.b_dof + in.m);
    P.b_sign.assign(in.b_sign, in.b_sign + in.m);
    P.dual_map.assign(in.dual_map, in.dual_map + in.m);
    for (int32_t j = 0; j < in.m; ++j) {
        if (P.b_dof[j] < 0 || P.b_dof[j] >= in.n) { P.err = "b_dof out of range"; return false; }
        if (P.b_sign[j] != 1 && P.b_sign[j] != -1) { P.err = "b_sign must be +1 or -1"; return false; }
        if (P.dual_map[j] < 0 || P.dual_map[j] >= n_lambda) { P.err = "dual_map out of range"; return false; }
        if (j > 0 && P.dual_map[j] <= P.dual_map[j - 1]) { P.err = "dual_map not strictly increasing"; return false; }
    }
    if (in.nelem > 0) {
        if (!in.elem_dofs || !in.dK || in.edofs <= 0) { P.err = "element data incomplete"; return false; }
        P.nelem = in.nelem;
        P.edofs = in.edofs;
        P.elem_dofs.assign(in.elem_dofs, in.elem_dofs + (size_t)in.nelem * in.edofs);
        P.dK.assign(in.dK, in.dK + (size_t)in.edofs * in.edofs);
        for (int32_t v : P.elem_dofs)
            if (v < 0 || v >= in.n) { P.err = "elem_dofs out of range"; return false; }
    }
    if (in.nkernel > 0) {
        if (in.nkernel > COARSE_MAXK || !in.R) { P.err = "nkernel must be <= 6 with R given"; return false; }
        P.nk = in.nkernel;
        P.R.assign(in.R, in.R + (size_t)in.n * in.nkernel);
    }
    SymbolicOptions so;
    so.leaf_nodes = opt.leaf_nodes;
    std::vector<char> last;
    if (opt.schur_order) {
        if (!multiplier_nodes(in, last)) { P.err = "b_dof out of range"; return false; }
        so.last_nodes = &last;
    }
    int dim = (in.coords && in.dim > 0) ? in.dim : 0;
    if (!symbolic_analysis(A, in.dofs_per_node, dim ? in.coords : nullptr, dim, so, P.sym, P.err)) return false;
    const Symbolic& S = P.sym;
    // RHS columns sorted by their start row (= by start supernode, postorder)
    std::vector<std::pair<int32_t, int32_t>> key(in.m);
    for (int32_t j = 0; j < in.m; ++j) key[j] = {S.pinv[P.b_dof[j]], j};
    std::stable_sort(key.begin(), key.end());
    P.sigma.resize(in.m);
    P.start.resize(in.m);
    for (int32_t k = 0; k < in.m; ++k) {
        P.sigma[k] = key[k].second;
        P.start[k] = key[k].first;
    }
    const int32_t ns = (int32_t)S.sn.size();
    std::vector<int32_t> fd(ns);
    for (int32_t s = 0; s < ns; ++s) fd[s] = S.sn[s].first;
    for (int32_t s = 0; s < ns; ++s)
        if (S.sn[s].parent >= 0) fd[S.sn[s].parent] = std::min(fd[S.sn[s].parent], fd[s]);
    P.j0.resize(ns);
    P.w.resize(ns);
    P.xoff.resize(ns);
    int64_t xo = 0;
    for (int32_t s = 0; s < ns; ++s) {
        int32_t a = (int32_t)(std::lower_bound(P.start.begin(), P.start.end(), fd[s]) - P.start.begin());
        int32_t b = (int32_t)(std::lower_bound(P.start.begin(), P.start.end(), S.sn[s].first + S.sn[s].ncols) -
                              P.start.begin());
        P.j0[s] = a;
        P.w[s] = b - a;
        P.xoff[s] = xo;
        xo += (int64_t)S.sn[s].ncols * P.w[s];
    }
    P.nx = xo;
    // lumped preconditioner tables
    std::vector<int32_t> bpos(in.n, -1);
    P.lb_mb.resize(in.m);
    P.lb_ms.resize(in.m);
    for (int32_t k = 0; k < in.m; ++k) {
        const int32_t dof = P.b_dof[P.sigma[k]];
        if (bpos[dof] < 0) {
            bpos[dof] = (int32_t)P.lb_dofs.size();
            P.lb_dofs.push_back(dof);
        }
        P.lb_mb[k] = bpos[dof];
        P.lb_ms[k] = P.b_sign[P.sigma[k]];
    }
    const int32_t nb = (int32_t)P.lb_dofs.size();
    P.lb_uptr.assign(nb + 1, 0);
    for (int32_t k = 0; k < in.m; ++k) P.lb_uptr[P.lb_mb[k] + 1]++;
    for (int32_t u = 0; u < nb; ++u) P.lb_uptr[u + 1] += P.lb_uptr[u];
    P.lb_uk.resize(in.m);
    {
        std::vector<int32_t> fill(P.lb_uptr.begin(), P.lb_uptr.end() - 1);
        for (int32_t k = 0; k < in.m; ++k) P.lb_uk[fill[P.lb_mb[k]]++] = k;
    }
    P.lb_kptr.assign(nb + 1, 0);
    P.lb_kdiag.assign(nb, -1);
    for (int32_t u = 0; u < nb; ++u) {
        const int32_t row = P.lb_dofs[u];
        for (int64_t e = A.ptr[row]; e < A.ptr[row + 1]; ++e)
            if (bpos[A.idx[e]] >= 0) {
                if (A.idx[e] == row) P.lb_kdiag[u] = (int32_t)P.lb_kcol.size();
                P.lb_kcol.push_back(bpos[A.idx[e]]);
                P.lb_ksrc.push_back(e);
            }
        P.lb_kptr[u + 1] = (int32_t)P.lb_kcol.size();
        if (P.lb_kdiag[u] < 0) { P.err = "pattern lacks the diagonal of a boundary DOF"; return false; }
    }
    return true;
}

}  // namespace

// ======================================================================== apply plan

namespace {

// The MI355X has 8 dies (XCDs), each with its own L2, and hands out the
// work-groups of a launch round-robin by index (index p to die p % 8).
// Work that re-reads the same data (the X rows and L panels of one
// subdomain) should share a die.  xcd_order gives every group (the items of
// one subdomain) one die -- largest groups first onto the least loaded die
// -- keeps each die's items in group order, and places the k-th item of die
// x at index k * kXcds + x; short queues are padded with `noop`.
constexpr int kXcds = 8;

template <typename T>
std::vector<T> xcd_order(const std::vector<std::vector<T>>& groups, const std::vector<double>& gcost, const T& noop)
{
    std::vector<size_t> ord(groups.size());
    for (size_t g = 0; g < ord.size(); ++g) ord[g] = g;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return gcost[a] > gcost[b]; });
    std::vector<std::vector<T>> q(kXcds);
    std::vector<double> load(kXcds, 0.0);
    std::vector<size_t> qn(kXcds, 0);
    for (size_t g : ord) {
        if (groups[g].empty()) continue;
        int best = 0;
        for (int x = 1; x < kXcds; ++x)
            if (load[x] < load[best] || (load[x] == load[best] && qn[x] < qn[best])) best = x;
        q[best].insert(q[best].end(), groups[g].begin(), groups[g].end());
        load[best] += gcost[g];
        qn[best] = q[best].size();
    }
    size_t L = 0;
    for (const auto& v : q) L = std::max(L, v.size());
    std::vector<T> out(L * kXcds, noop);
    for (int x = 0; x < kXcds; ++x)
        for (size_t k = 0; k < q[x].size(); ++k) out[k * kXcds + x] = q[x][k];
    return out;
}

struct ApplyPlan {
    std::vector<Band> bands;      // bands of rows, in subdomain order (indexed by the gather map)
    std::vector<Band> launch;     // the same bands in launch order
    std::vector<int32_t> seg_ptr; // work-group g handles launch[seg_ptr[g] .. seg_ptr[g+1])
    std::vector<int64_t> band_z;
    std::vector<int32_t> gptr;
    std::vector<int32_t> zptr;    // global multiplier g sums z[zpos[zptr[g] .. zptr[g+1])]
    std::vector<int64_t> zpos;
    int64_t total_z = 0;
};

// Work decomposition of the apply.  split 0: every triangle is cut into
// ceil(E_i / band_elems) bands of whole rows with about equal stored
// elements, one band per work-group, launched largest first so the short
// bands fill the tail.  split 1: the stored elements of all triangles,
// concatenated in subdomain order, are cut into G = total / band_elems equal
// shares (rows kept whole), one per work-group; a share is cut at subdomain
// boundaries into bands that its work-group handles in turn.  The gather map
// lists, for every global multiplier, its (subdomain, row) entries in
// ascending subdomain order with the bands whose partials hold that row.
void plan_apply(fetiF_ctx c, int32_t band_elems, int32_t split, ApplyPlan& A)
{
    const int V = prec_row_align(c->prec);
    band_elems = std::max(1, band_elems);
    int64_t total = 0;
    for (int32_t i = 0; i < c->nsub; ++i) total += packed_row_offset(c->subs[i].m, V);
    // first row of subdomain plan P starting at or after local element offset t
    auto cut_row = [&](const SubPlan& P, int64_t t) {
        int32_t lo = 0, hi = P.m;
        while (lo < hi) {
            int32_t mid = (lo + hi) / 2;
            if (packed_row_offset(mid, V) >= t) hi = mid;
            else lo = mid + 1;
        }
        return lo;
    };
    const int64_t G = split ? std::max<int64_t>(1, (total + band_elems / 2) / band_elems) : 0;
    // share g covers global element offsets [S(g), S(g+1))
    auto S = [&](int64_t g) { return (int64_t)((__int128)total * g / G); };
    auto share_of = [&](int64_t x) {
        int64_t g = std::min<int64_t>(G - 1, (int64_t)((__int128)x * G / std::max<int64_t>(1, total)));
        while (g + 1 < G && S(g + 1) <= x) ++g;
        while (g > 0 && S(g) > x) --g;
        return g;
    };
    int64_t zb = 0, off = 0;
    std::vector<int64_t> band_group;
    for (int32_t i = 0; i < c->nsub; ++i) {
        SubPlan& P = c->subs[i];
        const int64_t E = packed_row_offset(P.m, V);
        P.band0 = (int32_t)A.bands.size();
        std::vector<int32_t> cuts{0};
        if (split) {
            for (int64_t g = share_of(off) + 1; g < G && S(g) < off + E; ++g) {
                const int32_t r = cut_row(P, S(g) - off);
                if (r > cuts.back() && r < P.m) cuts.push_back(r);
            }
        } else {
            const int64_t nb = std::max<int64_t>(1, (E + band_elems - 1) / band_elems);
            for (int64_t k = 1; k < nb; ++k) {
                const int32_t r = cut_row(P, E * k / nb);
                if (r > cuts.back() && r < P.m) cuts.push_back(r);
            }
        }
        cuts.push_back(P.m);
        // at most kMaxBandRows rows per band (the segmented kernel keeps a
        // band's row scalars and sums in LDS): long stretches cut evenly
        {
            std::vector<int32_t> capped{0};
            for (size_t k = 1; k < cuts.size(); ++k) {
                const int32_t a0 = capped.back(), a1 = cuts[k];
                const int32_t np = (a1 - a0 + kMaxBandRows - 1) / kMaxBandRows;
                for (int32_t t = 1; t < np; ++t) capped.push_back(a0 + (int32_t)((int64_t)(a1 - a0) * t / np));
                capped.push_back(a1);
            }
            cuts.swap(capped);
        }
        for (size_t k = 0; k + 1 < cuts.size(); ++k) {
            const int32_t r0 = cuts[k], r1 = cuts[k + 1];
            if (r1 <= r0) continue;
            Band bd;
            bd.fbase = P.fbase;
            bd.zoff = zb;
            bd.r0 = r0;
            bd.r1 = r1;
            bd.dbase = P.dbase;
            bd.pad = 0;
            A.bands.push_back(bd);
            A.band_z.push_back(zb);
            if (split) band_group.push_back(share_of(off + packed_row_offset(r0, V)));
            zb += r1;
        }
        P.nband = (int32_t)A.bands.size() - P.band0;
        off += E;
    }
    A.total_z = zb;
    const int64_t nb = (int64_t)A.bands.size();
    if (split) {
        A.launch = A.bands;
        A.seg_ptr.assign(G + 1, 0);
        for (int64_t grp : band_group) A.seg_ptr[grp + 1]++;
        for (int64_t g = 0; g < G; ++g) A.seg_ptr[g + 1] += A.seg_ptr[g];
    } else {
        auto elems = [&](const Band& bd) { return packed_row_offset(bd.r1, V) - packed_row_offset(bd.r0, V); };
        std::vector<int64_t> order(nb);
        for (int64_t k = 0; k < nb; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t x, int64_t y) { return elems(A.bands[x]) > elems(A.bands[y]); });
        A.launch.resize(nb);
        for (int64_t k = 0; k < nb; ++k) A.launch[k] = A.bands[order[k]];
        A.seg_ptr.resize(nb + 1);
        for (int64_t k = 0; k <= nb; ++k) A.seg_ptr[k] = (int32_t)k;
    }
    // gather map: local row a of a subdomain receives the partial sums of
    // the subdomain's bands from the one holding row a to its last one (each
    // band's partial vector covers its columns 0 .. r1); multiplier g adds
    // its (subdomain, row) terms in ascending subdomain order, bands in
    // order.  Stored flat as positions in the partial vectors.
    const int64_t nl = c->n_lambda;
    std::vector<int64_t> cnt(nl + 1, 0);
    for (int32_t i = 0; i < c->nsub; ++i) {
        const SubPlan& P = c->subs[i];
        int32_t bcur = P.band0;
        for (int32_t a = 0; a < P.m; ++a) {
            while (A.bands[bcur].r1 <= a) ++bcur;
            cnt[P.dual_map[P.sigma[a]] + 1] += P.band0 + P.nband - bcur;
        }
    }
    int64_t total_terms = 0;
    for (int64_t g = 1; g <= nl; ++g) total_terms += cnt[g];
    if (total_terms > INT32_MAX) {   // not representable: install_apply refuses the plan
        A.zptr.clear();
        return;
    }
    A.zptr.assign(nl + 1, 0);
    for (int64_t g = 0; g < nl; ++g) A.zptr[g + 1] = A.zptr[g] + (int32_t)cnt[g + 1];
    A.zpos.resize(A.zptr[nl]);
    std::vector<int32_t> fill(A.zptr.begin(), A.zptr.end() - 1);
    for (int32_t i = 0; i < c->nsub; ++i) {
        const SubPlan& P = c->subs[i];
        int32_t bcur = P.band0;
        for (int32_t a = 0; a < P.m; ++a) {
            while (A.bands[bcur].r1 <= a) ++bcur;
            int32_t& f = fill[P.dual_map[P.sigma[a]]];
            for (int32_t bb = bcur; bb < P.band0 + P.nband; ++bb) A.zpos[f++] = A.band_z[bb] + a;
        }
    }
}

void free_apply(fetiF_ctx c)
{
    for (void* p : c->apply_allocs) (void)hipFree(p);
    c->apply_allocs.clear();
    c->dZ = nullptr;
    c->dBands = nullptr;
    c->dSegPtr = nullptr;
    c->ngroups = 0;
    c->dZptr = nullptr;
    c->dZpos = nullptr;
}

template <typename T>
hipError_t aalloc(fetiF_ctx c, T** p, size_t count)
{
    *p = nullptr;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(1, count));
    if (e == hipSuccess) {
        c->apply_allocs.push_back(q);
        *p = (T*)q;
    }
    return e;
}

// Device copies of an apply plan (replacing the previous one).
hipError_t install_apply(fetiF_ctx c, const ApplyPlan& A)
{
    free_apply(c);
    hipError_t e;
    char* z = nullptr;
    if ((e = aalloc(c, &z, (size_t)A.total_z * (c->prec == 0 ? 8 : 4) + 64)) != hipSuccess) return e;
    c->dZ = z;
    if ((e = aalloc(c, &c->dBands, A.launch.size())) != hipSuccess) return e;
    if ((e = aalloc(c, &c->dSegPtr, A.seg_ptr.size())) != hipSuccess) return e;
    if ((e = upload(c->dSegPtr, A.seg_ptr)) != hipSuccess) return e;
    c->ngroups = (int32_t)A.seg_ptr.size() - 1;
    if (A.zptr.empty()) return hipErrorInvalidValue;   // more gather terms than int32 indexes
    if ((e = aalloc(c, &c->dZptr, A.zptr.size())) != hipSuccess) return e;
    if ((e = aalloc(c, &c->dZpos, A.zpos.size())) != hipSuccess) return e;
    if ((e = upload(c->dBands, A.launch)) != hipSuccess) return e;
    if ((e = upload(c->dZptr, A.zptr)) != hipSuccess) return e;
    if ((e = upload(c->dZpos, A.zpos)) != hipSuccess) return e;
    c->nbands = (int32_t)A.bands.size();
    c->total_z = A.total_z;
    c->hZptr = A.zptr;
    c->hZpos = A.zpos;
    c->apply_brmax = 0;
    for (const Band& bd : A.bands) c->apply_brmax = std::max(c->apply_brmax, bd.r1 - bd.r0);
    return hipSuccess;
}

}  // namespace

// ======================================================================== TRSM plan

namespace {

struct TrsmPlan {
    std::vector<DevSN> tsns;        // column panels
    std::vector<int64_t> troff;     // X offset minus range start of every panel below row
    std::vector<TrsmItem> items;    // all levels, level by level
    std::vector<int64_t> level_off;
    std::vector<int32_t> level_waves, level_maxns;
};

// Assembly groups: contiguous subdomain ranges of about equal factor size
// (at most G of them, each of at least one subdomain per host thread so the
// group's factorisation keeps every thread busy); first[g] .. first[g+1] is
// group g.
std::vector<int32_t> plan_groups(fetiF_ctx c, int32_t G)
{
    G = std::max(1, std::min(G, c->nsub / std::max(1, c->nthreads)));
    int64_t total = 0;
    for (int32_t i = 0; i < c->nsub; ++i) total += c->subs[i].sym.nvals;
    std::vector<int32_t> first{0};
    int64_t acc = 0;
    for (int32_t i = 0; i + 1 < c->nsub; ++i) {
        acc += c->subs[i].sym.nvals;
        const int32_t g = (int32_t)first.size();   // index of the next group
        if (g < G && (double)acc * G >= (double)total * g && c->nsub - (i + 1) >= G - g) first.push_back(i + 1);
    }
    first.push_back(c->nsub);
    return first;
}

// TRSM schedule.  Every supernode with RHS columns is cut into column panels
// of at most `panel` columns (a multiple of 16): panel k starts at diagonal
// offset o = k * panel of the same storage, and the supernode's columns after
// the panel count among its below rows, so the panel's update of them is an
// ordinary below-row update.  Panel levels: panel k of a supernode runs one
// level after panel k - 1, and its first panel one level after the last
// panel of every child.  Two panels of one level then never belong to an
// ancestor and a descendant, so they own disjoint RHS column ranges and
// write disjoint entries of X.  A work-group has W wavefronts of 16 RHS
// columns each (W = chunk / 16, shrunk when the solved blocks, W *
// ceil(ncols/16) * 2 KiB of LDS, would not fit).
bool plan_trsm(fetiF_ctx c, int32_t panel, int32_t chunk, TrsmPlan& T)
{
    std::vector<int32_t> tlevel, tsub;
    int32_t tmaxlev = 0;
    for (int32_t i = 0; i < c->nsub; ++i) {
        const SubPlan& P = c->subs[i];
        const Symbolic& S = P.sym;
        const int32_t nsn = (int32_t)S.sn.size();
        std::vector<int32_t> next_level(nsn, 0);   // first level free above each supernode's panels
        for (int32_t s = 0; s < nsn; ++s) {        // postorder: children before parents
            const Supernode& x = S.sn[s];
            const DevSN& d = c->hSN[P.snbase + s];
            int32_t L = next_level[s];
            if (P.w[s] > 0) {
                for (int32_t o = 0; o < x.ncols; o += panel) {
                    const int32_t cw = std::min(panel, x.ncols - o);
                    DevSN t = d;
                    t.lval = d.lval + (int64_t)o * d.ld + o;
                    t.linv = d.linv + (int64_t)(o / 16) * 256;
                    t.xoff = d.xoff + (int64_t)o * P.w[s];
                    t.rowsoff = (int64_t)T.troff.size();
                    t.first = x.first + o;
                    t.ncols = cw;
                    t.nrows = x.ncols - o - cw + x.nrows;
                    for (int32_t k = o + cw; k < x.ncols; ++k) T.troff.push_back(c->hRowOff[P.rowbase + x.first + k]);
                    for (int32_t k = 0; k < x.nrows; ++k)
                        T.troff.push_back(c->hRowOff[P.rowbase + S.rows[x.row_off + k]]);
                    T.tsns.push_back(t);
                    tsub.push_back(i);
                    tlevel.push_back(L++);
                }
            }
            if (x.parent >= 0) next_level[x.parent] = std::max(next_level[x.parent], L);
            tmaxlev = std::max(tmaxlev, L - 1);
        }
    }
    std::vector<std::vector<TrsmItem>> lv(tmaxlev + 1);
    T.level_maxns.assign(tmaxlev + 1, 0);
    T.level_waves.assign(tmaxlev + 1, 4);
    for (size_t t = 0; t < T.tsns.size(); ++t)
        T.level_maxns[tlevel[t]] = std::max(T.level_maxns[tlevel[t]], T.tsns[t].ncols);
    const int32_t wmax = std::max(1, std::min(4, chunk / 16));
    // a level whose panels mostly have few RHS columns gets narrower
    // work-groups (more of them per CU): W covers 90 % of its panels' widths
    std::vector<std::vector<int32_t>> lw(tmaxlev + 1);
    for (size_t t = 0; t < T.tsns.size(); ++t) lw[tlevel[t]].push_back(T.tsns[t].w);
    for (int32_t L = 0; L <= tmaxlev; ++L) {
        const int32_t mx = std::max(1, T.level_maxns[L]);
        int32_t W = wmax;
        if (!lw[L].empty()) {
            std::vector<int32_t>& v = lw[L];
            const size_t k = (v.size() * 9) / 10;
            std::nth_element(v.begin(), v.begin() + (ptrdiff_t)std::min(k, v.size() - 1), v.end());
            const int32_t w90 = v[std::min(k, v.size() - 1)];
            while (W > 1 && 16 * (W / 2) >= w90) W /= 2;
        }
        while (W > 1 && trsm_lds_bytes(W, mx) > 80 * 1024) W /= 2;   // keep two work-groups per CU
        if (trsm_lds_bytes(W, mx) > 160 * 1024) return false;
        T.level_waves[L] = W;
    }
    for (size_t t = 0; t < T.tsns.size(); ++t) {
        const int32_t L = tlevel[t];
        const int32_t slot = 16 * T.level_waves[L];
        for (int32_t c0 = 0; c0 < T.tsns[t].w; c0 += slot) {
            TrsmItem it;
            it.sn = (int32_t)t;
            it.c0 = c0;
            it.cw = std::min(slot, T.tsns[t].w - c0);
            it.pad = 0;
            lv[L].push_back(it);
        }
    }
    // per level: the items of a subdomain on one die (they share its L
    // panels and X rows), larger panels first
    auto icost = [&](const TrsmItem& a) {
        const DevSN& x = T.tsns[a.sn];
        return (double)x.ncols * (x.ncols + 2.0 * x.nrows) * a.cw;
    };
    TrsmItem noop{};
    noop.cw = 0;   // no columns: the kernel returns at once
    // items ordered by assembly group, then level: group g's level L is
    // items [level_off[g * nlev + L], level_off[g * nlev + L + 1])
    const int32_t G = (int32_t)c->grp_first.size() - 1;
    const int32_t nlev = tmaxlev + 1;
    T.level_off.assign((size_t)G * nlev + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
        const int32_t s0 = c->grp_first[g], s1 = c->grp_first[g + 1];
        for (int32_t L = 0; L < nlev; ++L) {
            std::vector<std::vector<TrsmItem>> per_sub(s1 - s0);
            std::vector<double> sub_cost(s1 - s0, 0.0);
            for (const TrsmItem& it : lv[L]) {
                const int32_t i = tsub[it.sn];
                if (i < s0 || i >= s1) continue;
                per_sub[i - s0].push_back(it);
                sub_cost[i - s0] += icost(it);
            }
            for (auto& v : per_sub)
                std::stable_sort(v.begin(), v.end(), [&](const TrsmItem& a, const TrsmItem& b) {
                    const DevSN& x = T.tsns[a.sn];
                    const DevSN& y = T.tsns[b.sn];
                    return (int64_t)x.ncols * (x.ncols + 2 * x.nrows) > (int64_t)y.ncols * (y.ncols + 2 * y.nrows);
                });
            const std::vector<TrsmItem> v = xcd_order(per_sub, sub_cost, noop);
            T.level_off[(size_t)g * nlev + L] = (int64_t)T.items.size();
            T.items.insert(T.items.end(), v.begin(), v.end());
        }
    }
    T.level_off[(size_t)G * nlev] = (int64_t)T.items.size();
    return true;
}

void free_trsm(fetiF_ctx c)
{
    for (void* p : c->trsm_allocs) (void)hipFree(p);
    c->trsm_allocs.clear();
    c->dTSN = nullptr;
    c->dTRowOff = nullptr;
    c->dItems = nullptr;
}

template <typename T>
hipError_t talloc(fetiF_ctx c, T** p, size_t count)
{
    *p = nullptr;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(1, count));
    if (e == hipSuccess) {
        c->trsm_allocs.push_back(q);
        *p = (T*)q;
    }
    return e;
}

// Device copies of a TRSM plan (replacing the previous one).
hipError_t install_trsm(fetiF_ctx c, const TrsmPlan& T)
{
    free_trsm(c);
    hipError_t e;
    if ((e = talloc(c, &c->dTSN, T.tsns.size())) != hipSuccess) return e;
    if ((e = talloc(c, &c->dTRowOff, T.troff.size())) != hipSuccess) return e;
    if ((e = talloc(c, &c->dItems, T.items.size())) != hipSuccess) return e;
    if ((e = upload(c->dTSN, T.tsns)) != hipSuccess) return e;
    if ((e = upload(c->dTRowOff, T.troff)) != hipSuccess) return e;
    if ((e = upload(c->dItems, T.items)) != hipSuccess) return e;
    c->level_off = T.level_off;
    c->level_waves = T.level_waves;
    c->level_maxns = T.level_maxns;
    c->trsm_levels = (int32_t)T.level_waves.size();
    return hipSuccess;
}

void free_bwd(fetiF_ctx c)
{
    for (void* p : c->bwd_allocs) (void)hipFree(p);
    c->bwd_allocs.clear();
    c->dZfull = nullptr;
    c->dBPan = nullptr;
    c->dBZrow = nullptr;
    c->dBItems = nullptr;
    c->dZbase = nullptr;
    c->dFbase = nullptr;
    c->blevel_off.clear();
    c->total_zfull = 0;
    c->trsm_bwd_flops = 0;
}

template <typename T>
hipError_t balloc(fetiF_ctx c, T** p, size_t count)
{
    *p = nullptr;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * std::max<size_t>(1, count));
    if (e == hipSuccess) {
        c->bwd_allocs.push_back(q);
        *p = (T*)q;
    }
    return e;
}

// Plan and device tables of the TRSM path's backward solve (Sec. IV-C):
// column panels of at most `panel` columns of every supernode of every
// subdomain (Z is dense, so supernodes without RHS columns take part too),
// levelled like the forward panels (a supernode's panels in a chain, a
// parent above its children) and run from the top level down; one item per
// 64 of the subdomain's m_i columns.  Z_i is n_i x m_i row-major.
hipError_t install_bwd(fetiF_ctx c, int32_t panel)
{
    free_bwd(c);
    std::vector<DevSN> pans;
    std::vector<int64_t> zrow, zbase(c->nsub), fbase(c->nsub);
    std::vector<int32_t> plevel;
    int32_t maxlev = 0;
    int64_t zb = 0;
    double flops = 0;
    for (int32_t i = 0; i < c->nsub; ++i) {
        const SubPlan& P = c->subs[i];
        const Symbolic& S = P.sym;
        zbase[i] = zb;
        fbase[i] = P.fbase;
        const int32_t nsn = (int32_t)S.sn.size();
        std::vector<int32_t> next_level(nsn, 0);
        auto zoff = [&](int32_t row) { return zb + (int64_t)row * P.m; };
        for (int32_t s = 0; s < nsn; ++s) {
            const Supernode& x = S.sn[s];
            const DevSN& d = c->hSN[P.snbase + s];
            int32_t L = next_level[s];
            for (int32_t o = 0; o < x.ncols; o += panel) {
                const int32_t cw = std::min(panel, x.ncols - o);
                DevSN t = d;
                t.lval = d.lval + (int64_t)o * d.ld + o;
                t.linv = d.linv + (int64_t)(o / 16) * 256;
                t.xoff = d.xoff + (int64_t)o * P.w[s];
                t.rowsoff = (int64_t)zrow.size();
                t.first = x.first + o;
                t.ncols = cw;
                t.nrows = x.ncols - o - cw + x.nrows;
                t.pad = P.m;
                for (int32_t k = o; k < x.ncols; ++k) zrow.push_back(zoff(x.first + k));
                for (int32_t k = 0; k < x.nrows; ++k) zrow.push_back(zoff(S.rows[x.row_off + k]));
                flops += ((double)cw * cw + 2.0 * cw * t.nrows) * P.m;
                pans.push_back(t);
                plevel.push_back(L++);
            }
            if (x.parent >= 0) next_level[x.parent] = std::max(next_level[x.parent], L);
            maxlev = std::max(maxlev, L - 1);
        }
        zb += (int64_t)P.n * P.m;
    }
    // items, level by level (within a level, subdomain by subdomain)
    std::vector<std::vector<TrsmItem>> lv(maxlev + 1);
    for (size_t t = 0; t < pans.size(); ++t)
        for (int32_t c0 = 0; c0 < pans[t].pad; c0 += 64) {
            TrsmItem it;
            it.sn = (int32_t)t;
            it.c0 = c0;
            it.cw = std::min(64, pans[t].pad - c0);
            it.pad = 0;
            lv[plevel[t]].push_back(it);
        }
    std::vector<TrsmItem> items;
    c->blevel_off.assign(maxlev + 2, 0);
    for (int32_t L = 0; L <= maxlev; ++L) {
        c->blevel_off[L] = (int64_t)items.size();
        items.insert(items.end(), lv[L].begin(), lv[L].end());
    }
    c->blevel_off[maxlev + 1] = (int64_t)items.size();
    hipError_t e;
    if ((e = balloc(c, &c->dZfull, (size_t)zb)) != hipSuccess) return e;
    if ((e = balloc(c, &c->dBPan, pans.size())) != hipSuccess) return e;
    if ((e = balloc(c, &c->dBZrow, zrow.size())) != hipSuccess) return e;
    if ((e = balloc(c, &c->dBItems, items.size())) != hipSuccess) return e;
    if ((e = balloc(c, &c->dZbase, zbase.size())) != hipSuccess) return e;
    if ((e = balloc(c, &c->dFbase, fbase.size())) != hipSuccess) return e;
    if ((e = upload(c->dBPan, pans)) != hipSuccess) return e;
    if ((e = upload(c->dBZrow, zrow)) != hipSuccess) return e;
    if ((e = upload(c->dBItems, items)) != hipSuccess) return e;
    if ((e = upload(c->dZbase, zbase)) != hipSuccess) return e;
    if ((e = upload(c->dFbase, fbase)) != hipSuccess) return e;
    c->total_zfull = zb;
    c->trsm_bwd_flops = flops;
    return hipSuccess;
}

// The TRSM path after the forward solve: backward levels from the top
// down, then the SpMM F~ = B~ P^T Z into the packed triangles.
hipError_t trsm_path_tail(fetiF_ctx c, hipStream_t st)
{
    const int32_t nlev = (int32_t)c->blevel_off.size() - 1;
    {
        PhaseTimer t7(c, st, 7);
        for (int32_t L = nlev - 1; L >= 0; --L) {
            const int32_t cnt = (int32_t)(c->blevel_off[L + 1] - c->blevel_off[L]);
            hipError_t e = launch_trsm_bwd_level(c->dBItems + c->blevel_off[L], cnt, 4, c->dBPan, c->dL, c->dLinv,
                                                 c->dBZrow, c->dX, c->dZfull, st);
            if (e != hipSuccess) return e;
        }
        hipError_t e = t7.stop();
        if (e != hipSuccess) return e;
    }
    PhaseTimer t8(c, st, 8);
    hipError_t e = launch_tri_from_z(c->prec, c->nsub, c->sum_m, c->dSubM, c->dStartRows, c->dSignsSorted, c->dZbase,
                                     c->dFbase, c->dZfull, c->dF, st);
    if (e != hipSuccess) return e;
    return t8.stop();
}

}  // namespace

// ======================================================================== create

extern "C" fetiF_status fetiF_create(fetiF_ctx* out, int device, int64_t n_lambda, int32_t nsub,
                                     const fetiF_subdomain* subs, const fetiF_options* opt_in)
{
    if (!out) return fail(nullptr, FETIF_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsub <= 0 || !subs || n_lambda <= 0 || n_lambda > INT32_MAX)
        return fail(nullptr, FETIF_EINVAL, "need nsub > 0, subs, 0 < n_lambda < 2^31");
    fetiF_options opt;
    options_defaults(opt_in, opt);
    if (opt.f_storage < FETIF_F64 || opt.f_storage > FETIF_BF16) return fail(nullptr, FETIF_EINVAL, "bad f_storage");
    fetiF_ctx c = new (std::nothrow) fetiF_ctx_s();
    if (!c) return fail(nullptr, FETIF_ENOMEM, "host allocation failed");
    c->device = device;
    c->n_lambda = n_lambda;
    c->nsub = nsub;
    c->opt = opt;
    c->prec = (int)opt.f_storage;
    // default: the CPUs this process may run on (the affinity mask), not
    // every CPU of the machine
    unsigned hc = 0;
    {
        cpu_set_t cs;
        CPU_ZERO(&cs);
        if (sched_getaffinity(0, sizeof(cs), &cs) == 0) hc = (unsigned)CPU_COUNT(&cs);
        if (!hc) hc = std::thread::hardware_concurrency();
    }
    c->nthreads = opt.nthreads > 0 ? opt.nthreads : (int)(hc ? hc : 1);
    c->subs.resize(nsub);

    // ---- per-subdomain analysis on host threads
    parallel_for(nsub, c->nthreads, [&](int32_t i) {
        if (!plan_subdomain(subs[i], opt, n_lambda, c->subs[i]))
            if (c->subs[i].err.empty()) c->subs[i].err = "analysis failed";
    });
    for (int32_t i = 0; i < nsub; ++i)
        if (!c->subs[i].err.empty()) {
            std::string msg = "subdomain " + std::to_string(i) + ": " + c->subs[i].err;
            delete c;
            return fail(nullptr, FETIF_EINVAL, msg);
        }

    const int V = prec_vec(c->prec), RA = prec_row_align(c->prec);
    const int TS = 64;
    // ---- global placement and schedules
    std::vector<DevSN> sns;
    std::vector<InvItem> inv_items;
    int64_t linv_b = 0;
    std::vector<int32_t> rows;
    std::vector<XRow> xrows;
    std::vector<RhsUnit> units;
    std::vector<SyrkTile> tiles;
    std::vector<int32_t> lists;
    std::vector<int32_t> dmap;
    int64_t lb = 0, xb = 0, fb = 0;
    int32_t snb = 0, rowb = 0, db = 0;
    int32_t maxlev = 0, max_m = 0;
    for (int32_t i = 0; i < nsub; ++i) {
        SubPlan& P = c->subs[i];
        const Symbolic& S = P.sym;
        P.lbase = lb;
        P.xbase = xb;
        P.snbase = snb;
        P.inv0 = (int32_t)inv_items.size();
        P.rowbase = rowb;
        P.dbase = db;
        const int32_t ns = (int32_t)S.sn.size();
        for (int32_t s = 0; s < ns; ++s) {
            const Supernode& x = S.sn[s];
            // the TRSM reads a panel (at most 96 of the supernode's columns,
            // each of ld = ncols + nrows entries) through 32-bit byte offsets
            if ((int64_t)std::min<int32_t>(x.ncols, 96) * (x.ncols + x.nrows) * 8 > INT32_MAX) {
                delete c;
                return fail(nullptr, FETIF_ENOTSUP, "a supernode's panel exceeds 2^31 bytes");
            }
            DevSN d;
            d.lval = lb + x.val_off;
            {
                d.linv = linv_b;
                const int32_t nbk = (x.ncols + 15) / 16;
                for (int32_t rb = 0; rb < nbk; ++rb) inv_items.push_back({snb + s, rb});
                linv_b += (int64_t)nbk * 256;
            }
            d.xoff = xb + P.xoff[s];
            d.rowsoff = (int64_t)rows.size();
            d.rowbase = rowb;
            d.first = x.first;
            d.ncols = x.ncols;
            d.nrows = x.nrows;
            d.j0 = P.j0[s];
            d.w = P.w[s];
            d.ld = x.ncols + x.nrows;
            d.pad = 0;
            sns.push_back(d);
            rows.insert(rows.end(), S.rows.begin() + x.row_off, S.rows.begin() + x.row_off + x.nrows);
            maxlev = std::max(maxlev, x.level);
            c->trsm_flops += ((double)x.ncols * x.ncols + 2.0 * x.ncols * x.nrows) * P.w[s];
            c->syrk_flops += (double)x.ncols * P.w[s] * (P.w[s] + 1);
        }
        c->factor_flops += S.flops_factor;
        P.ninv = (int32_t)inv_items.size() - P.inv0;
        xrows.resize(xrows.size() + P.n);
        for (int32_t s = 0; s < ns; ++s) {
            const Supernode& x = S.sn[s];
            for (int32_t k = 0; k < x.ncols; ++k) {
                XRow& r = xrows[rowb + x.first + k];
                r.off = xb + P.xoff[s] + (int64_t)k * P.w[s];
                r.j0 = P.j0[s];
                r.w = P.w[s];
            }
        }
        for (int32_t k = 0; k < P.m; ++k) {
            const XRow& r = xrows[rowb + P.start[k]];
            RhsUnit u;
            u.off = r.off + (k - r.j0);
            u.sign = (double)P.b_sign[P.sigma[k]];
            units.push_back(u);
            dmap.push_back(P.dual_map[P.sigma[k]]);
        }
        // F storage and SYRK tiles
        P.fbase = fb;
        const int64_t fel = packed_row_offset(P.m, RA);
        const int32_t nt = (P.m + TS - 1) / TS;
        for (int32_t ta = 0; ta < nt; ++ta)
            for (int32_t tb = 0; tb <= ta; ++tb) {
                SyrkTile t;
                t.fbase = fb;
                t.m = P.m;
                t.ta = ta;
                t.tb = tb;
                t.list0 = (int32_t)lists.size();
                for (int32_t s = 0; s < ns; ++s) {
                    if (P.w[s] <= 0) continue;
                    int32_t a = P.j0[s], b = P.j0[s] + P.w[s];
                    if (a < std::min((tb + 1) * TS, P.m) && b > ta * TS) lists.push_back(snb + s);
                }
                t.list1 = (int32_t)lists.size();
                t.pad = 0;
                tiles.push_back(t);
            }
        max_m = std::max(max_m, P.m);
        lb += S.nvals;
        xb += P.nx;
        fb += fel + 64;  // a little slack keeps the tail of every triangle aligned
        snb += ns;
        rowb += P.n;
        db += P.m;
        c->sum_m += P.m;
    }
    c->total_L = lb;
    c->total_X = xb;
    c->total_F = fb;
    c->total_rows = rowb;
    c->nsyrk = (int32_t)tiles.size();
    // chunk count of the whole-row apply kernel (lanes cover NCH * 64 * V
    // columns, all held in LDS): 0 when the largest subdomain is too wide for
    // it, and then the column-segmented kernel, which holds any m, serves
    {
        int nch = 1;
        while ((int64_t)nch * 64 * V < max_m) nch *= 2;
        c->apply_nch = (int64_t)nch * 64 * V > kMaxWholeRowCols ? 0 : nch;
        c->max_m = max_m;
        if (c->apply_nch == 0 && c->opt.apply_seg == 0) c->opt.apply_seg = 4;
    }
    // host copies the TRSM planner needs again when it re-plans
    c->hSN = sns;
    c->hRowOff.resize(xrows.size());
    for (size_t r = 0; r < xrows.size(); ++r) c->hRowOff[r] = xrows[r].off - xrows[r].j0;
    c->grp_first = plan_groups(c, opt.assembly_groups);
    const int32_t ngrp = (int32_t)c->grp_first.size() - 1;
    TrsmPlan tplan;
    if (!plan_trsm(c, opt.trsm_panel, opt.trsm_chunk, tplan)) {
        delete c;
        return fail(nullptr, FETIF_ENOTSUP, "TRSM panel does not fit in LDS");
    }
    // SYRK tiles: the tiles of a subdomain on one die, most expensive first
    {
        std::vector<std::vector<SyrkTile>> per_sub(nsub);
        std::vector<double> sub_cost(nsub, 0.0);
        auto tcost = [&](const SyrkTile& t) {
            int64_t cst = 0;
            for (int32_t li = t.list0; li < t.list1; ++li) cst += sns[lists[li]].ncols;
            return cst;
        };
        for (size_t t = 0, i = 0; t < tiles.size(); ++t) {
            while (i + 1 < (size_t)nsub && tiles[t].fbase != c->subs[i].fbase) ++i;  // made subdomain by subdomain
            per_sub[i].push_back(tiles[t]);
            sub_cost[i] += (double)tcost(tiles[t]);
        }
        for (auto& v : per_sub)
            std::stable_sort(v.begin(), v.end(),
                             [&](const SyrkTile& a, const SyrkTile& b) { return tcost(a) > tcost(b); });
        SyrkTile noop{};
        noop.m = 0;   // no output: the kernel returns at once
        // group by group: group g's tiles are [syrk_off[g], syrk_off[g+1])
        tiles.clear();
        c->syrk_off.assign(ngrp + 1, 0);
        for (int32_t g = 0; g < ngrp; ++g) {
            const int32_t s0 = c->grp_first[g], s1 = c->grp_first[g + 1];
            const std::vector<std::vector<SyrkTile>> gs(per_sub.begin() + s0, per_sub.begin() + s1);
            const std::vector<double> gc(sub_cost.begin() + s0, sub_cost.begin() + s1);
            const std::vector<SyrkTile> v = xcd_order(gs, gc, noop);
            c->syrk_off[g] = (int64_t)tiles.size();
            tiles.insert(tiles.end(), v.begin(), v.end());
        }
        c->syrk_off[ngrp] = (int64_t)tiles.size();
        c->nsyrk = (int32_t)tiles.size();
    }
    ApplyPlan aplan;
    plan_apply(c, opt.apply_band, opt.apply_split, aplan);

    // ---- tables of the batched solves with L
    std::vector<int32_t> relpos(rows.size(), -1), child_ptr(sns.size() + 1, 0), child_idx;
    std::vector<int32_t> sub_row(nsub + 1, 0), sub_m(nsub + 1, 0), start_rows, xperm;
    std::vector<int8_t> signs_sorted;
    c->solve_levels.assign(maxlev + 1, {});
    c->solve_maxfront.assign(maxlev + 1, 1);
    {
        std::vector<std::vector<int32_t>> kids(sns.size());
        for (int32_t i = 0; i < nsub; ++i) {
            const SubPlan& P = c->subs[i];
            const Symbolic& S = P.sym;
            std::vector<int32_t> pos(P.n, -1);
            for (size_t sl = 0; sl < S.sn.size(); ++sl) {
                const Supernode& x = S.sn[sl];
                const int32_t g = P.snbase + (int32_t)sl;
                c->solve_levels[x.level].push_back(g);
                c->solve_maxfront[x.level] = std::max(c->solve_maxfront[x.level], x.ncols + x.nrows);
                if (x.parent < 0) continue;
                kids[P.snbase + x.parent].push_back(g);
                const Supernode& p = S.sn[x.parent];
                for (int32_t k = 0; k < p.ncols; ++k) pos[p.first + k] = k;
                for (int32_t k = 0; k < p.nrows; ++k) pos[S.rows[p.row_off + k]] = p.ncols + k;
                for (int32_t k = 0; k < x.nrows; ++k) {
                    int32_t pr = pos[S.rows[x.row_off + k]];
                    if (pr < 0) {
                        delete c;
                        return fail(nullptr, FETIF_EINVAL, "internal: child rows outside the parent front");
                    }
                    relpos[sns[g].rowsoff + k] = pr;
                }
                for (int32_t k = 0; k < p.ncols; ++k) pos[p.first + k] = -1;
                for (int32_t k = 0; k < p.nrows; ++k) pos[S.rows[p.row_off + k]] = -1;
            }
            sub_row[i + 1] = sub_row[i] + P.n;
            sub_m[i + 1] = sub_m[i] + P.m;
            for (int32_t k = 0; k < P.m; ++k) {
                start_rows.push_back(P.start[k]);
                signs_sorted.push_back(P.b_sign[P.sigma[k]]);
            }
            for (int32_t k = 0; k < P.n; ++k) xperm.push_back(P.rowbase + S.perm[k]);
        }
        for (size_t g = 0; g < sns.size(); ++g) {
            child_ptr[g + 1] = child_ptr[g] + (int32_t)kids[g].size();
            child_idx.insert(child_idx.end(), kids[g].begin(), kids[g].end());
        }
    }
    std::vector<int32_t> solve_sn;
    c->solve_off.assign(maxlev + 2, 0);
    for (int32_t L = 0; L <= maxlev; ++L) {
        c->solve_off[L] = (int64_t)solve_sn.size();
        solve_sn.insert(solve_sn.end(), c->solve_levels[L].begin(), c->solve_levels[L].end());
    }
    c->solve_off[maxlev + 1] = (int64_t)solve_sn.size();
    c->total_u = (int64_t)rows.size();
    // implicit gather: global multiplier -> (x position, sign), ascending subdomain
    std::vector<int32_t> xgptr(n_lambda + 1, 0);
    for (int32_t i = 0; i < nsub; ++i)
        for (int32_t g : c->subs[i].dual_map) xgptr[g + 1]++;
    for (int64_t g = 0; g < n_lambda; ++g) xgptr[g + 1] += xgptr[g];
    std::vector<XGatherEnt> xgent(xgptr[n_lambda]);
    {
        std::vector<int32_t> fill(xgptr.begin(), xgptr.end() - 1);
        for (int32_t i = 0; i < nsub; ++i) {
            const SubPlan& P = c->subs[i];
            for (int32_t j = 0; j < P.m; ++j) {
                XGatherEnt e;
                e.xpos = P.rowbase + P.sym.pinv[P.b_dof[j]];
                e.sign = (double)P.b_sign[j];
                xgent[fill[P.dual_map[j]]++] = e;
            }
        }
    }
    // element tables of the theta-adjoint
    std::vector<ElemRef> elems;
    std::vector<int32_t> epos;
    std::vector<double> dks;
    c->has_elems = true;
    for (int32_t i = 0; i < nsub; ++i)
        if (c->subs[i].nelem <= 0) c->has_elems = false;
    if (c->has_elems) {
        for (int32_t i = 0; i < nsub; ++i) {
            const SubPlan& P = c->subs[i];
            const int64_t dko = (int64_t)dks.size();
            dks.insert(dks.end(), P.dK.begin(), P.dK.end());
            for (int32_t e = 0; e < P.nelem; ++e) {
                ElemRef r;
                r.sub = i;
                r.edofs = P.edofs;
                r.pos_off = (int64_t)epos.size();
                r.dk_off = dko;
                for (int32_t a = 0; a < P.edofs; ++a)
                    epos.push_back(P.rowbase + P.sym.pinv[P.elem_dofs[(size_t)e * P.edofs + a]]);
                elems.push_back(r);
            }
        }
        c->nelem_total = (int64_t)elems.size();
    }

    // coarse space G = B R (sorted multiplier order) and G^T G
    std::vector<CoarseSub> csub;
    std::vector<double> gvals, Rcat, GtG;
    std::vector<int32_t> g2ptr;
    std::vector<GEnt> g2ent;
    c->has_coarse = true;
    for (int32_t i = 0; i < nsub; ++i)
        if (c->subs[i].nk <= 0) c->has_coarse = false;
    if (c->has_coarse) {
        int32_t koff = 0;
        int64_t rbs = 0;
        for (int32_t i = 0; i < nsub; ++i) {
            SubPlan& P = c->subs[i];
            P.koff = koff;
            CoarseSub cs;
            cs.mbase = P.dbase;
            cs.gvbase = 0;
            cs.rbase = rbs;
            cs.m = P.m;
            cs.nk = P.nk;
            cs.koff = koff;
            cs.n = P.n;
            cs.rowbase = P.rowbase;
            cs.pad = 0;
            csub.push_back(cs);
            for (int32_t a = 0; a < P.m; ++a) {
                const int32_t j = P.sigma[a];
                for (int32_t k = 0; k < P.nk; ++k)
                    gvals.push_back((double)P.b_sign[j] * P.R[(size_t)P.b_dof[j] * P.nk + k]);
            }
            Rcat.insert(Rcat.end(), P.R.begin(), P.R.end());
            koff += P.nk;
            rbs += P.n;
        }
        c->ncoarse = koff;
        // rows of G per global multiplier, ascending subdomain; gvals rows are
        // laid out with each subdomain's own nk, so keep explicit offsets
        std::vector<int64_t> gvoff(nsub + 1, 0);
        for (int32_t i = 0; i < nsub; ++i) gvoff[i + 1] = gvoff[i] + (int64_t)c->subs[i].m * c->subs[i].nk;
        g2ptr.assign(n_lambda + 1, 0);
        for (int32_t i = 0; i < nsub; ++i)
            for (int32_t g : c->subs[i].dual_map) g2ptr[g + 1]++;
        for (int64_t g = 0; g < n_lambda; ++g) g2ptr[g + 1] += g2ptr[g];
        g2ent.resize(g2ptr[n_lambda]);
        {
            std::vector<int32_t> fill(g2ptr.begin(), g2ptr.end() - 1);
            for (int32_t i = 0; i < nsub; ++i) {
                const SubPlan& P = c->subs[i];
                for (int32_t a = 0; a < P.m; ++a) {
                    GEnt e;
                    e.gv = gvoff[i] + (int64_t)a * P.nk;
                    e.koff = P.koff;
                    e.nk = P.nk;
                    g2ent[fill[P.dual_map[P.sigma[a]]]++] = e;
                }
            }
        }
        for (int32_t i = 0; i < nsub; ++i) csub[i].gvbase = gvoff[i];
        const int64_t nc = c->ncoarse;
        GtG.assign((size_t)nc * nc, 0.0);
        for (int64_t g = 0; g < n_lambda; ++g)
            for (int32_t e1 = g2ptr[g]; e1 < g2ptr[g + 1]; ++e1)
                for (int32_t e2 = g2ptr[g]; e2 < g2ptr[g + 1]; ++e2) {
                    const GEnt& A1 = g2ent[e1];
                    const GEnt& A2 = g2ent[e2];
                    for (int32_t k1 = 0; k1 < A1.nk; ++k1)
                        for (int32_t k2 = 0; k2 < A2.nk; ++k2)
                            GtG[(size_t)(A1.koff + k1) * nc + A2.koff + k2] += gvals[A1.gv + k1] * gvals[A2.gv + k2];
                }
    }

    // ---- device memory
    {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
            delete c;
            return fail(nullptr, FETIF_EDEVICE, "no HIP device available");
        }
        if (device < 0 || device >= ndev) {
            delete c;
            return fail(nullptr, FETIF_EINVAL, "device ordinal out of range");
        }
    }
    DeviceGuard dg(device);
    if (!dg.ok) {
        delete c;
        return fail(nullptr, FETIF_EDEVICE, "hipSetDevice failed");
    }
    auto bail = [&](hipError_t e, const char* what) {
        fetiF_status st = hip_fail(nullptr, e, what);
        for (void* p : c->allocations) (void)hipFree(p);
        c->allocations.clear();
        free_apply(c);
        free_trsm(c);
        if (c->hStage) (void)hipHostFree(c->hStage);
        delete c;
        return st;
    };
#define CK(call)                                   \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return bail(e_, #call); \
    } while (0)
    // the device address of the static scratch of fetiF_apply_static, looked
    // up here once per device (with the device current)
    CK(static_scratch_address(device, &c->dScratch));
    if (c->opt.debug_checks) CK(dalloc(c, &c->dDbg, 1));
    CK(dalloc(c, &c->dL, (size_t)c->total_L));
    CK(dalloc(c, &c->dX, (size_t)c->total_X));
    {
        char* f = nullptr;
        CK(dalloc(c, &f, (size_t)c->total_F * prec_bytes(c->prec) + 64));
        c->dF = f;
        CK(hipMemset(f, 0, (size_t)c->total_F * prec_bytes(c->prec) + 64));
    }
    c->total_linv = linv_b;
    c->ninv = (int32_t)inv_items.size();
    CK(dalloc(c, &c->dLinv, (size_t)linv_b));
    CK(dalloc(c, &c->dInv, inv_items.size()));
    CK(upload(c->dInv, inv_items));
    CK(dalloc(c, &c->dSolveSn, solve_sn.size()));
    CK(upload(c->dSolveSn, solve_sn));
    CK(dalloc(c, &c->dChildPtr, child_ptr.size()));
    CK(upload(c->dChildPtr, child_ptr));
    CK(dalloc(c, &c->dChildIdx, child_idx.size()));
    CK(upload(c->dChildIdx, child_idx));
    CK(dalloc(c, &c->dRelpos, relpos.size()));
    CK(upload(c->dRelpos, relpos));
    CK(dalloc(c, &c->dU, (size_t)c->total_u * 2));
    CK(dalloc(c, &c->dXv, (size_t)c->total_rows * 2));
    CK(dalloc(c, &c->dSubRow, sub_row.size()));
    CK(upload(c->dSubRow, sub_row));
    CK(dalloc(c, &c->dSubM, sub_m.size()));
    CK(upload(c->dSubM, sub_m));
    CK(dalloc(c, &c->dStartRows, start_rows.size()));
    CK(upload(c->dStartRows, start_rows));
    CK(dalloc(c, &c->dSignsSorted, signs_sorted.size()));
    CK(upload(c->dSignsSorted, signs_sorted));
    CK(dalloc(c, &c->dXGptr, xgptr.size()));
    CK(upload(c->dXGptr, xgptr));
    CK(dalloc(c, &c->dXGent, xgent.size()));
    CK(upload(c->dXGent, xgent));
    CK(dalloc(c, &c->dXperm, xperm.size()));
    CK(upload(c->dXperm, xperm));
    if (c->has_elems) {
        CK(dalloc(c, &c->dElems, elems.size()));
        CK(upload(c->dElems, elems));
        CK(dalloc(c, &c->dEpos, epos.size()));
        CK(upload(c->dEpos, epos));
        CK(dalloc(c, &c->dDK, dks.size()));
        CK(upload(c->dDK, dks));
    }
    if (c->has_coarse) {
        const int64_t nc = c->ncoarse;
        CK(dalloc(c, &c->dCoarse, csub.size()));
        CK(upload(c->dCoarse, csub));
        CK(dalloc(c, &c->dGv, gvals.size()));
        CK(upload(c->dGv, gvals));
        CK(dalloc(c, &c->dGptr2, g2ptr.size()));
        CK(upload(c->dGptr2, g2ptr));
        CK(dalloc(c, &c->dGent2, g2ent.size()));
        CK(upload(c->dGent2, g2ent));
        CK(dalloc(c, &c->dR, Rcat.size()));
        CK(upload(c->dR, Rcat));
        CK(dalloc(c, &c->dAinv, (size_t)(nc * nc)));
        CK(upload(c->dAinv, GtG));
        CK(dalloc(c, &c->dVec, (size_t)(9 * n_lambda)));
        // lumped preconditioner tables (global slots; see LumpSub)
        {
            std::vector<LumpSub> ls(nsub);
            std::vector<int32_t> uptr{0}, uk, kptr{0}, kcol, mb(c->sum_m), gptr(n_lambda + 1, 0), gpos(c->sum_m);
            std::vector<double> sg(c->sum_m);
            int32_t bb = 0;
            int64_t kb = 0;
            for (int32_t i = 0; i < nsub; ++i) {
                SubPlan& P = c->subs[i];
                const int32_t nb = (int32_t)P.lb_dofs.size();
                ls[i] = LumpSub{bb, nb, P.dbase, P.m};
                P.lb_kbase = kb;
                for (int32_t u = 0; u < nb; ++u) {
                    uptr.push_back(P.dbase + P.lb_uptr[u + 1]);
                    kptr.push_back((int32_t)(kb + P.lb_kptr[u + 1]));
                }
                for (int32_t e = 0; e < P.m; ++e) uk.push_back(P.dbase + P.lb_uk[e]);
                for (int32_t v : P.lb_kcol) kcol.push_back(bb + v);
                for (int32_t k = 0; k < P.m; ++k) {
                    mb[P.dbase + k] = bb + P.lb_mb[k];
                    sg[P.dbase + k] = P.lb_ms[k];
                    gptr[P.dual_map[P.sigma[k]] + 1]++;
                }
                bb += nb;
                kb += (int64_t)P.lb_kcol.size();
                c->lb_nbmax = std::max(c->lb_nbmax, nb);
            }
            if (kb > INT32_MAX) {
                delete c;
                return fail(nullptr, FETIF_ENOTSUP, "lumped preconditioner tables exceed 2^31 entries");
            }
            for (int64_t g = 0; g < n_lambda; ++g) gptr[g + 1] += gptr[g];
            {
                std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
                for (int32_t i = 0; i < nsub; ++i) {   // ascending subdomain order per multiplier
                    const SubPlan& P = c->subs[i];
                    for (int32_t k = 0; k < P.m; ++k) gpos[fill[P.dual_map[P.sigma[k]]]++] = P.dbase + k;
                }
            }
            c->lb_nk = kb;
            CK(dalloc(c, &c->dLump, ls.size()));
            CK(upload(c->dLump, ls));
            CK(dalloc(c, &c->dLbUptr, uptr.size()));
            CK(upload(c->dLbUptr, uptr));
            CK(dalloc(c, &c->dLbUk, uk.size()));
            CK(upload(c->dLbUk, uk));
            CK(dalloc(c, &c->dLbKptr, kptr.size()));
            CK(upload(c->dLbKptr, kptr));
            CK(dalloc(c, &c->dLbKcol, kcol.size()));
            CK(upload(c->dLbKcol, kcol));
            CK(dalloc(c, &c->dLbMb, mb.size()));
            CK(upload(c->dLbMb, mb));
            CK(dalloc(c, &c->dLbSgn, sg.size()));
            CK(upload(c->dLbSgn, sg));
            CK(dalloc(c, &c->dLbGptr, gptr.size()));
            CK(upload(c->dLbGptr, gptr));
            CK(dalloc(c, &c->dLbGpos, gpos.size()));
            CK(upload(c->dLbGpos, gpos));
            CK(dalloc(c, &c->dLbKval, (size_t)std::max<int64_t>(1, kb)));
            CK(dalloc(c, &c->dLbY, (size_t)c->sum_m));
            // groups of multipliers coupled through a shared (subdomain, DOF):
            // the diagonal blocks of A = B W B^T (union-find over multipliers)
            {
                std::vector<int32_t> uf((size_t)n_lambda);
                for (int64_t g = 0; g < n_lambda; ++g) uf[(size_t)g] = (int32_t)g;
                auto root = [&](int32_t x) {
                    while (uf[(size_t)x] != x) {
                        uf[(size_t)x] = uf[(size_t)uf[(size_t)x]];
                        x = uf[(size_t)x];
                    }
                    return x;
                };
                for (int32_t i = 0; i < nsub; ++i) {
                    const SubPlan& P = c->subs[i];
                    for (size_t u = 0; u + 1 < P.lb_uptr.size(); ++u)
                        for (int32_t e = P.lb_uptr[u] + 1; e < P.lb_uptr[u + 1]; ++e) {
                            const int32_t a = root(P.dual_map[P.sigma[P.lb_uk[P.lb_uptr[u]]]]);
                            const int32_t b = root(P.dual_map[P.sigma[P.lb_uk[e]]]);
                            if (a != b) uf[(size_t)std::max(a, b)] = std::min(a, b);
                        }
                }
                std::vector<int32_t> bid((size_t)n_lambda, -1);
                c->hSbOf.assign((size_t)n_lambda, 0);
                c->hSbPos.assign((size_t)n_lambda, 0);
                std::vector<int32_t> cnt;
                for (int64_t g = 0; g < n_lambda; ++g) {   // blocks numbered by their smallest member
                    const int32_t r = root((int32_t)g);
                    if (bid[(size_t)r] < 0) {
                        bid[(size_t)r] = (int32_t)cnt.size();
                        cnt.push_back(0);
                    }
                    c->hSbOf[(size_t)g] = bid[(size_t)r];
                    c->hSbPos[(size_t)g] = cnt[(size_t)bid[(size_t)r]]++;
                }
                const size_t nbk = cnt.size();
                c->hSbPtr.assign(nbk + 1, 0);
                c->hSbOff.assign(nbk + 1, 0);
                for (size_t b = 0; b < nbk; ++b) {
                    c->hSbPtr[b + 1] = c->hSbPtr[b] + cnt[b];
                    c->hSbOff[b + 1] = c->hSbOff[b] + (int64_t)cnt[b] * cnt[b];
                }
                c->hSbMem.assign((size_t)n_lambda, 0);
                for (int64_t g = 0; g < n_lambda; ++g)
                    c->hSbMem[(size_t)(c->hSbPtr[(size_t)c->hSbOf[(size_t)g]] + c->hSbPos[(size_t)g])] = (int32_t)g;
                CK(dalloc(c, &c->dSbOf, c->hSbOf.size()));
                CK(upload(c->dSbOf, c->hSbOf));
                CK(dalloc(c, &c->dSbPos, c->hSbPos.size()));
                CK(upload(c->dSbPos, c->hSbPos));
                CK(dalloc(c, &c->dSbPtr, c->hSbPtr.size()));
                CK(upload(c->dSbPtr, c->hSbPtr));
                CK(dalloc(c, &c->dSbMem, c->hSbMem.size()));
                CK(upload(c->dSbMem, c->hSbMem));
                CK(dalloc(c, &c->dSbOff, c->hSbOff.size()));
                CK(upload(c->dSbOff, c->hSbOff));
                CK(dalloc(c, &c->dSbInv, (size_t)std::max<int64_t>(1, c->hSbOff.back())));
                CK(dalloc(c, &c->dLbCoef, (size_t)c->sum_m));
                c->lb_given.assign((size_t)nsub, 0);
            }
            CK(hipHostMalloc((void**)&c->hLbKval, sizeof(double) * (size_t)std::max<int64_t>(1, kb),
                             hipHostMallocDefault));
        }
        CK(dalloc(c, &c->dCvec, (size_t)(3 * nc + 2 * nc)));
        CK(dalloc(c, &c->dPart, (size_t)2 * dot_parts(c->n_lambda)));
        CK(dalloc(c, &c->dSc, (size_t)SC_COUNT + 8));
        // scalars and the dot kernel's completion counter (after SC_COUNT) start at zero
        CK(hipMemset(c->dSc, 0, sizeof(double) * ((size_t)SC_COUNT + 8)));
        // (G^T G)^{-1} in place by Gauss-Jordan steps on the device; the two
        // trailing coarse vectors serve as the pivot row/column buffers
        CK(launch_gauss_jordan_inverse((int32_t)nc, c->dAinv, c->dCvec + 3 * nc, c->dCvec + 4 * nc, nullptr));
    }
    CK(dalloc(c, &c->dSN, sns.size()));
    CK(dalloc(c, &c->dRows, rows.size()));
    CK(dalloc(c, &c->dXRows, xrows.size()));
    CK(dalloc(c, &c->dUnits, units.size()));
    CK(dalloc(c, &c->dTiles, tiles.size()));
    CK(dalloc(c, &c->dLists, lists.size()));
    CK(dalloc(c, &c->dDmap, dmap.size()));
    CK(upload(c->dSN, sns));
    CK(upload(c->dRows, rows));
    CK(upload(c->dXRows, xrows));
    CK(upload(c->dUnits, units));
    CK(install_trsm(c, tplan));
    CK(upload(c->dTiles, tiles));
    CK(upload(c->dLists, lists));
    CK(upload(c->dDmap, dmap));
    c->hDmap = dmap;
    CK(install_apply(c, aplan));
    CK(hipHostMalloc((void**)&c->hStage, sizeof(double) * (size_t)std::max<int64_t>(1, c->total_L),
                     hipHostMallocDefault));
    CK(hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming));
    CK(hipDeviceSynchronize());
#undef CK
    c->uploaded.assign(nsub, 0);
    *out = c;
    return FETIF_OK;
}

// ======================================================================== factor + upload

namespace {

// Host factorisation of subdomains [first, first+count) and the asynchronous
// copy of their values on st (no wait for earlier copies: every subdomain has
// its own staging area).  Chunks of at least 64 MiB of factor values and of
// at least 4 subdomains per host thread, but no more than a quarter of the
// range (a shorter rest joins the last chunk): the copy of a chunk and its
// diagonal-block inverses run on the stream while the host factors the next
// chunk.  With `one_chunk` the whole range is one chunk (an assembly group,
// whose copy and assembly already overlap the factorisation of the next
// group).  Within a chunk the threads take the subdomains largest
// factorisation first, so that uneven subdomains still end together.
fetiF_status upload_range(fetiF_ctx c, int32_t first, int32_t count, const double* const* k_vals, hipStream_t st,
                          bool one_chunk = false)
{
    // any upload replaces factor values: F~ must be assembled again, and on
    // failure the whole range counts as not uploaded
    c->assembled = false;
    constexpr int64_t kChunkVals = int64_t(8) << 20;
    const int32_t min_subs = one_chunk ? count : std::max(c->nthreads, std::min(4 * c->nthreads, count / 4));
    for (int32_t k0 = 0; k0 < count;) {
        int32_t k1 = k0;
        int64_t vals = 0;
        while (k1 < count && (k1 - k0 < min_subs || vals < kChunkVals)) vals += c->subs[first + k1++].sym.nvals;
        if (count - k1 < min_subs) k1 = count;
        std::vector<int32_t> bad(k1 - k0, -1);
        std::vector<int32_t> order(k1 - k0);
        for (int32_t k = 0; k < k1 - k0; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return c->subs[first + k0 + a].sym.flops_factor > c->subs[first + k0 + b].sym.flops_factor;
        });
        parallel_for(k1 - k0, c->nthreads, [&](int32_t kk) {
            const int32_t k = order[kk];
            const SubPlan& P = c->subs[first + k0 + k];
            bad[k] = numeric_cholesky(P.sym, k_vals[k0 + k], c->hStage + P.lbase);
            // the K_reg entries among boundary DOFs, for the lumped
            // preconditioners (unless fetiF_precond_values gave other values)
            if (c->hLbKval && !c->lb_given[(size_t)(first + k0 + k)])
                for (size_t e = 0; e < P.lb_ksrc.size(); ++e) c->hLbKval[P.lb_kbase + e] = k_vals[k0 + k][P.lb_ksrc[e]];
        });
        for (int32_t k = 0; k < k1 - k0; ++k)
            if (bad[k] >= 0) {
                const SubPlan& P = c->subs[first + k0 + k];
                for (int32_t t = 0; t < count; ++t)
                    if (c->uploaded[first + t]) {
                        c->uploaded[first + t] = 0;
                        c->n_uploaded--;
                    }
                // earlier copies may still read the staging area
                HIPCHK(c, hipEventRecord(c->upload_done, st));
                c->upload_pending = true;
                return fail(c, FETIF_ENOTSPD,
                            "subdomain " + std::to_string(first + k0 + k) + ": non-positive pivot at permuted column " +
                                std::to_string(bad[k]) + " (original dof " + std::to_string(P.sym.perm[bad[k]]) + ")");
            }
        const SubPlan& P0 = c->subs[first + k0];
        const SubPlan& P1 = c->subs[first + k1 - 1];
        const int64_t n = P1.lbase + P1.sym.nvals - P0.lbase;
        PhaseTimer t0(c, st, 0);
        HIPCHK(c, hipMemcpyAsync(c->dL + P0.lbase, c->hStage + P0.lbase, sizeof(double) * (size_t)n,
                                 hipMemcpyHostToDevice, st));
        if (c->hLbKval) {
            c->sb_dirty = true;
            const int64_t kb0 = P0.lb_kbase, kb1 = P1.lb_kbase + (int64_t)P1.lb_ksrc.size();
            if (kb1 > kb0)
                HIPCHK(c, hipMemcpyAsync(c->dLbKval + kb0, c->hLbKval + kb0, sizeof(double) * (size_t)(kb1 - kb0),
                                         hipMemcpyHostToDevice, st));
        }
        // inverses of the 16x16 diagonal blocks of the uploaded supernodes,
        // used by the assembly TRSM and by the solves
        HIPCHK(c, launch_diag_inverse(c->dInv + P0.inv0, P1.inv0 + P1.ninv - P0.inv0, c->dSN, c->dL, c->dLinv, st));
        HIPCHK(c, t0.stop());
        k0 = k1;
    }
    HIPCHK(c, hipEventRecord(c->upload_done, st));
    c->upload_pending = true;
    for (int32_t k = 0; k < count; ++k)
        if (!c->uploaded[first + k]) {
            c->uploaded[first + k] = 1;
            c->n_uploaded++;
        }
    return FETIF_OK;
}

// The device work of one assembly group g (contiguous subdomains): RHS
// initialisation of its X, its TRSM levels, its SYRK tiles.
hipError_t rhs_group(fetiF_ctx c, int32_t g, hipStream_t st)
{
    const SubPlan& A = c->subs[c->grp_first[g]];
    const SubPlan& B = c->subs[c->grp_first[g + 1] - 1];
    hipError_t e = launch_fill_zero(c->dX + A.xbase, B.xbase + B.nx - A.xbase, st);
    if (e != hipSuccess) return e;
    return launch_rhs_units(c->dUnits + A.dbase, (int64_t)B.dbase + B.m - A.dbase, c->dX, st);
}

hipError_t trsm_group(fetiF_ctx c, int32_t g, hipStream_t st)
{
    const int32_t nlev = c->trsm_levels;
    for (int32_t L = 0; L < nlev; ++L) {
        const size_t k = (size_t)g * nlev + L;
        const int32_t cnt = (int32_t)(c->level_off[k + 1] - c->level_off[k]);
        hipError_t e = launch_trsm_level(c->dItems + c->level_off[k], cnt, c->level_waves[L], c->level_maxns[L],
                                         c->dTSN, c->dL, c->dLinv, c->dTRowOff, c->dX, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t syrk_group(fetiF_ctx c, int32_t g, hipStream_t st)
{
    return launch_syrk(c->prec, c->dTiles + c->syrk_off[g], (int32_t)(c->syrk_off[g + 1] - c->syrk_off[g]),
                       c->dLists, c->dSN, c->dX, c->dF, st);
}

}  // namespace

extern "C" fetiF_status fetiF_factor_upload(fetiF_ctx c, int32_t first, int32_t count,
                                            const double* const* k_vals, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (first < 0 || count <= 0 || first + count > c->nsub || !k_vals)
        return fail(c, FETIF_EINVAL, "subdomain range out of bounds or k_vals NULL");
    for (int32_t k = 0; k < count; ++k)
        if (!k_vals[k]) return fail(c, FETIF_EINVAL, "k_vals entry is NULL");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    // the staging area may still be read by the previous asynchronous copy
    if (c->upload_pending) {
        HIPCHK(c, hipEventSynchronize(c->upload_done));
        c->upload_pending = false;
    }
    return upload_range(c, first, count, k_vals, (hipStream_t)stream);
}

// ======================================================================== assemble

// Debug scan (option debug_checks): waits for the stream's work, then reports
// the first NaN or Inf among x[0, n) (elements of precision prec) as
// FETIF_ENONFINITE, naming the call and the vector.
static fetiF_status debug_scan(fetiF_ctx c, int prec, const void* x, int64_t n, const char* call, const char* what,
                        hipStream_t st)
{
    HIPCHK(c, launch_first_nonfinite(prec, x, n, c->dDbg, st));
    unsigned long long first = ~0ull;
    HIPCHK(c, hipMemcpyAsync(&first, c->dDbg, sizeof first, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (first != ~0ull)
        return fail(c, FETIF_ENONFINITE,
                    std::string(call) + ": " + what + " holds a NaN or Inf at index " + std::to_string(first));
    return FETIF_OK;
}


extern "C" fetiF_status fetiF_assemble(fetiF_ctx c, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (c->n_uploaded != c->nsub) return fail(c, FETIF_ESTATE, "assemble before every subdomain was factored and uploaded");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, order_after_upload(c, st));
    const int32_t G = (int32_t)c->grp_first.size() - 1;
    // phase by phase over the groups (one timer per phase)
    PhaseTimer t1(c, st, 1);
    for (int32_t g = 0; g < G; ++g) HIPCHK(c, rhs_group(c, g, st));
    HIPCHK(c, t1.stop());
    PhaseTimer t2(c, st, 2);
    for (int32_t g = 0; g < G; ++g) HIPCHK(c, trsm_group(c, g, st));
    HIPCHK(c, t2.stop());
    if (c->assembly_path == 1) {
        HIPCHK(c, trsm_path_tail(c, st));
    } else {
        PhaseTimer t3(c, st, 3);
        for (int32_t g = 0; g < G; ++g) HIPCHK(c, syrk_group(c, g, st));
        HIPCHK(c, t3.stop());
    }
    c->assembled = true;
    if (c->opt.debug_checks) return debug_scan(c, c->prec, c->dF, c->total_F, "fetiF_assemble", "the stored F~", st);
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_set_assembly_path(fetiF_ctx c, int32_t path)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (path != 0 && path != 1) return fail(c, FETIF_EINVAL, "path must be 0 (SYRK) or 1 (TRSM)");
    if (path == c->assembly_path) return FETIF_OK;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    HIPCHK(c, hipDeviceSynchronize());
    if (path == 1) {
        const hipError_t e = install_bwd(c, c->opt.trsm_panel);
        if (e == hipErrorOutOfMemory) {
            free_bwd(c);
            (void)hipGetLastError();
            return fail(c, FETIF_ENOMEM, "the TRSM path's dense Z (sum n_i m_i FP64 values) does not fit");
        }
        HIPCHK(c, e);
    } else {
        free_bwd(c);
    }
    c->assembly_path = path;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_factor_assemble(fetiF_ctx c, const double* const* k_vals, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (!k_vals) return fail(c, FETIF_EINVAL, "k_vals NULL");
    for (int32_t k = 0; k < c->nsub; ++k)
        if (!k_vals[k]) return fail(c, FETIF_EINVAL, "k_vals entry is NULL");
    if (c->assembly_path != 0)
        return fail(c, FETIF_ENOTSUP, "fetiF_factor_assemble runs the SYRK path only (set path 0, or use "
                                      "fetiF_factor_upload + fetiF_assemble)");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    if (c->upload_pending) {
        HIPCHK(c, hipEventSynchronize(c->upload_done));
        c->upload_pending = false;
    }
    const int32_t G = (int32_t)c->grp_first.size() - 1;
    for (int32_t g = 0; g < G; ++g) {
        const int32_t s0 = c->grp_first[g], s1 = c->grp_first[g + 1];
        fetiF_status s = upload_range(c, s0, s1 - s0, k_vals + s0, st, true);
        if (s != FETIF_OK) {
            // earlier groups were uploaded and assembled from this call's
            // values, later ones hold older factors: nothing counts as uploaded
            std::fill(c->uploaded.begin(), c->uploaded.end(), 0);
            c->n_uploaded = 0;
            c->assembled = false;
            return s;
        }
        // the group's assembly is enqueued behind its copy; the host goes on
        // to factor the next group meanwhile
        PhaseTimer t1(c, st, 1);
        HIPCHK(c, rhs_group(c, g, st));
        HIPCHK(c, t1.stop());
        PhaseTimer t2(c, st, 2);
        HIPCHK(c, trsm_group(c, g, st));
        HIPCHK(c, t2.stop());
        PhaseTimer t3(c, st, 3);
        HIPCHK(c, syrk_group(c, g, st));
        HIPCHK(c, t3.stop());
    }
    c->assembled = true;
    return FETIF_OK;
}

// ======================================================================== apply

namespace {

// Band kernel + gather of one apply, with the partial vectors in z.
fetiF_status apply_with_partials(fetiF_ctx c, const double* lambda_d, double* q_d, void* z, hipStream_t st)
{
    PhaseTimer t4(c, st, 4);
    if (c->opt.apply_seg > 0) {
        HIPCHK(c, launch_apply_seg(c->prec, c->opt.apply_seg, c->opt.apply_rows, c->opt.apply_nontemporal != 0,
                                   c->dBands, c->dSegPtr, c->ngroups, c->dF, lambda_d, c->dDmap, z,
                                   c->apply_brmax, st));
    } else {
        HIPCHK(c, launch_apply_band(c->prec, c->apply_nch, c->opt.apply_rows, c->opt.apply_nontemporal != 0,
                                    c->dBands, c->dSegPtr, c->ngroups, c->dF, lambda_d, c->dDmap, z, st));
    }
    HIPCHK(c, t4.stop());
    PhaseTimer t5(c, st, 5);
    HIPCHK(c, launch_gather(c->prec, c->n_lambda, c->dZptr, c->dZpos, z, q_d, st));
    HIPCHK(c, t5.stop());
    return FETIF_OK;
}

fetiF_status apply_checks(fetiF_ctx c, const double* lambda_d, const double* q_d)
{
    if (c->sticky) return FETIF_EDEVICE;
    if (!lambda_d || !q_d) return fail(c, FETIF_EINVAL, "lambda or q is NULL");
    if (lambda_d == q_d) return fail(c, FETIF_EINVAL, "lambda and q must not overlap");
    if (!c->assembled) return fail(c, FETIF_ESTATE, "apply before assemble");
    return FETIF_OK;
}

}  // namespace


extern "C" fetiF_status fetiF_apply(fetiF_ctx c, const double* lambda_d, double* q_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    const fetiF_status s0 = apply_checks(c, lambda_d, q_d);
    if (s0 != FETIF_OK) return s0;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    if (c->opt.debug_checks)
        if (fetiF_status s1 = debug_scan(c, 0, lambda_d, c->n_lambda, "fetiF_apply", "lambda", st)) return s1;
    const fetiF_status s2 = apply_with_partials(c, lambda_d, q_d, c->dZ, st);
    if (s2 != FETIF_OK || !c->opt.debug_checks) return s2;
    return debug_scan(c, 0, q_d, c->n_lambda, "fetiF_apply", "q", st);
}

extern "C" fetiF_status fetiF_apply_static(fetiF_ctx c, const double* lambda_d, double* q_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    const fetiF_status s0 = apply_checks(c, lambda_d, q_d);
    if (s0 != FETIF_OK) return s0;
    const size_t need = (size_t)c->total_z * (c->prec == 0 ? 8 : 4);
    if (need > kStaticScratchBytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "fetiF_apply_static: the apply partials need %zu bytes, the static scratch holds %zu "
                      "(use fetiF_apply, or fewer, larger apply bands)",
                      need, kStaticScratchBytes);
        return fail(c, FETIF_ENOTSUP, msg);
    }
    if (!c->dScratch) return fail(c, FETIF_ESTATE, "static scratch address not set");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    if (c->opt.debug_checks)
        if (fetiF_status s1 = debug_scan(c, 0, lambda_d, c->n_lambda, "fetiF_apply_static", "lambda", st)) return s1;
    const fetiF_status s2 = apply_with_partials(c, lambda_d, q_d, c->dScratch, st);
    if (s2 != FETIF_OK || !c->opt.debug_checks) return s2;
    return debug_scan(c, 0, q_d, c->n_lambda, "fetiF_apply_static", "q", st);
}

extern "C" fetiF_status fetiF_apply_host(fetiF_ctx c, const double* lambda_h, double* q_h, int32_t cpu_scatter_gather,
                                         void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (!lambda_h || !q_h) return fail(c, FETIF_EINVAL, "lambda or q is NULL");
    if (lambda_h == q_h) return fail(c, FETIF_EINVAL, "lambda and q must not overlap");
    if (cpu_scatter_gather != 0 && cpu_scatter_gather != 1) return fail(c, FETIF_EINVAL, "cpu_scatter_gather must be 0 or 1");
    if (!c->assembled) return fail(c, FETIF_ESTATE, "apply before assemble");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nl = c->n_lambda, sm = c->sum_m;
    const size_t zb = (size_t)c->total_z * (c->prec == 0 ? 8 : 4);
    // buffers on first use (and when a new apply plan needs more partials)
    if (!c->dHostVec) {
        HIPCHK(c, hipMalloc((void**)&c->dHostVec, sizeof(double) * (size_t)(2 * nl + sm)));
        std::vector<int32_t> id((size_t)sm);
        for (int64_t k = 0; k < sm; ++k) id[(size_t)k] = (int32_t)k;
        HIPCHK(c, hipMalloc((void**)&c->dDmapId, sizeof(int32_t) * (size_t)std::max<int64_t>(1, sm)));
        HIPCHK(c, hipMemcpy(c->dDmapId, id.data(), sizeof(int32_t) * (size_t)sm, hipMemcpyHostToDevice));
    }
    const size_t need = sizeof(double) * (size_t)(2 * nl + sm) + zb;
    if (c->hPinBytes < need) {
        if (c->hPin) HIPCHK(c, hipHostFree(c->hPin));
        c->hPin = nullptr;
        c->hPinBytes = 0;
        HIPCHK(c, hipHostMalloc((void**)&c->hPin, need, hipHostMallocDefault));
        c->hPinBytes = need;
    }
    double* dLam = c->dHostVec;
    double* dQ = dLam + nl;
    double* dP = dQ + nl;
    double* hLam = c->hPin;
    double* hQ = hLam + nl;
    double* hP = hQ + nl;
    void* hZ = hP + sm;
    if (cpu_scatter_gather == 0) {
        // the cluster-wide vector to the device, scatter, SYMV and gather
        // there, the result back
        std::memcpy(hLam, lambda_h, sizeof(double) * (size_t)nl);
        HIPCHK(c, hipMemcpyAsync(dLam, hLam, sizeof(double) * (size_t)nl, hipMemcpyHostToDevice, st));
        const fetiF_status s1 = apply_with_partials(c, dLam, dQ, c->dZ, st);
        if (s1 != FETIF_OK) return s1;
        HIPCHK(c, hipMemcpyAsync(hQ, dQ, sizeof(double) * (size_t)nl, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        std::memcpy(q_h, hQ, sizeof(double) * (size_t)nl);
        return FETIF_OK;
    }
    // scatter on the host threads into the subdomain vectors p~_i (sorted
    // local order, concatenated), one copy to the device, the band kernels
    // with the identity map, one copy of the band partials back, gather on
    // the host threads in the same fixed order as the gather kernel
    const int32_t nchunk = std::max(1, std::min<int32_t>(c->nthreads * 4, (int32_t)((sm + 4095) / 4096)));
    parallel_for(nchunk, c->nthreads, [&](int32_t k) {
        const int64_t a = sm * k / nchunk, b = sm * (k + 1) / nchunk;
        for (int64_t t = a; t < b; ++t) hP[t] = lambda_h[c->hDmap[(size_t)t]];
    });
    HIPCHK(c, hipMemcpyAsync(dP, hP, sizeof(double) * (size_t)sm, hipMemcpyHostToDevice, st));
    {
        PhaseTimer t4(c, st, 4);
        if (c->opt.apply_seg > 0) {
            HIPCHK(c, launch_apply_seg(c->prec, c->opt.apply_seg, c->opt.apply_rows, c->opt.apply_nontemporal != 0,
                                       c->dBands, c->dSegPtr, c->ngroups, c->dF, dP, c->dDmapId, c->dZ,
                                       c->apply_brmax, st));
        } else {
            HIPCHK(c, launch_apply_band(c->prec, c->apply_nch, c->opt.apply_rows, c->opt.apply_nontemporal != 0,
                                        c->dBands, c->dSegPtr, c->ngroups, c->dF, dP, c->dDmapId, c->dZ, st));
        }
        HIPCHK(c, t4.stop());
    }
    HIPCHK(c, hipMemcpyAsync(hZ, c->dZ, zb, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const int32_t gchunk = std::max(1, std::min<int32_t>(c->nthreads * 4, (int32_t)((nl + 4095) / 4096)));
    const bool f64 = c->prec == 0;
    parallel_for(gchunk, c->nthreads, [&](int32_t k) {
        const int64_t a = nl * k / gchunk, b = nl * (k + 1) / gchunk;
        for (int64_t g = a; g < b; ++g) {
            double acc = 0.0;
            for (int32_t t = c->hZptr[(size_t)g]; t < c->hZptr[(size_t)g + 1]; ++t) {
                const int64_t pos = c->hZpos[(size_t)t];
                acc += f64 ? ((const double*)hZ)[pos] : (double)((const float*)hZ)[pos];
            }
            q_h[g] = acc;
        }
    });
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_read_probe(const void* buf_d, int64_t bytes, int64_t region_bytes, double* out_d,
                                         void* stream)
{
    if (!buf_d || !out_d || bytes <= 0 || bytes % 16 != 0 || region_bytes <= 0 || region_bytes % 16384 != 0 ||
        (bytes + region_bytes - 1) / region_bytes > INT32_MAX)
        return fail(nullptr, FETIF_EINVAL, "fetiF_read_probe: buf and out set, bytes a positive multiple of 16, "
                                           "region a positive multiple of 16384");
    const hipError_t e = launch_read_probe(buf_d, bytes, region_bytes, out_d, (hipStream_t)stream);
    return e == hipSuccess ? FETIF_OK : hip_fail(nullptr, e, "read probe launch");
}

extern "C" fetiF_status fetiF_set_assembly(fetiF_ctx c, int32_t trsm_panel, int32_t trsm_chunk)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (trsm_panel < 0 || trsm_panel > 96 || trsm_panel % 16 != 0 ||
        (trsm_chunk != 0 && trsm_chunk != 16 && trsm_chunk != 32 && trsm_chunk != 64))
        return fail(c, FETIF_EINVAL, "trsm_panel a multiple of 16 in [16, 96] (0 keeps), trsm_chunk in {0,16,32,64}");
    const int32_t np = trsm_panel > 0 ? trsm_panel : c->opt.trsm_panel;
    const int32_t nc = trsm_chunk > 0 ? trsm_chunk : c->opt.trsm_chunk;
    if (np == c->opt.trsm_panel && nc == c->opt.trsm_chunk) return FETIF_OK;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    TrsmPlan T;
    if (!plan_trsm(c, np, nc, T)) return fail(c, FETIF_ENOTSUP, "TRSM panel does not fit in LDS");
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, install_trsm(c, T));
    if (c->assembly_path == 1 && np != c->opt.trsm_panel) HIPCHK(c, install_bwd(c, np));
    c->opt.trsm_panel = np;
    c->opt.trsm_chunk = nc;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_set_apply(fetiF_ctx c, int32_t band_elems, int32_t rows, int32_t nontemporal,
                                        int32_t split, int32_t seg)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (band_elems < 0 || (rows != 0 && rows != 2 && rows != 4) || nontemporal < -1 || nontemporal > 1 ||
        split < -1 || split > 1 || (seg != -1 && seg != 0 && seg != 2 && seg != 3 && seg != 4 && seg != 8))
        return fail(c, FETIF_EINVAL,
                    "band_elems >= 0, rows in {0,2,4}, nontemporal in {-1,0,1}, split in {-1,0,1}, "
                    "seg in {-1,0,2,3,4,8}");
    if (seg == 0 && c->apply_nch == 0)
        return fail(c, FETIF_ENOTSUP,
                    "the whole-row apply kernel holds at most " + std::to_string(kMaxWholeRowCols) +
                        " columns (largest m = " + std::to_string(c->max_m) + "): use seg 4 or 8");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    if (c->pcpg_graph) {
        HIPCHK(c, hipDeviceSynchronize());
        (void)hipGraphExecDestroy(c->pcpg_graph);
        c->pcpg_graph = nullptr;
        c->pcpg_graph_key = -1;
    }
    if (rows) c->opt.apply_rows = rows;
    if (nontemporal >= 0) c->opt.apply_nontemporal = nontemporal;
    if (seg >= 0) c->opt.apply_seg = seg;
    const int32_t nb = band_elems > 0 ? band_elems : c->opt.apply_band;
    const int32_t ns = split >= 0 ? split : c->opt.apply_split;
    if (nb != c->opt.apply_band || ns != c->opt.apply_split) {
        HIPCHK(c, hipDeviceSynchronize());
        ApplyPlan A;
        plan_apply(c, nb, ns, A);
        HIPCHK(c, install_apply(c, A));
        c->opt.apply_band = nb;
        c->opt.apply_split = ns;
    }
    return FETIF_OK;
}

// Forward and backward substitution with every L_i on the nrhs vectors held
// in c->dXv (permuted rows, interleaved).
hipError_t fetif::solve_all(fetiF_ctx c, int nrhs, hipStream_t st)
{
    hipError_t e;
    const int32_t nl = (int32_t)c->solve_levels.size();
    for (int32_t L = 0; L < nl; ++L) {
        const int32_t n = (int32_t)(c->solve_off[L + 1] - c->solve_off[L]);
        if ((e = launch_trsv_forward_level(nrhs, c->dSolveSn + c->solve_off[L], n, c->solve_maxfront[L], c->dSN, c->dL,
                                           c->dLinv, c->dChildPtr, c->dChildIdx, c->dRelpos, c->dU, c->dXv, st)) !=
            hipSuccess)
            return e;
    }
    for (int32_t L = nl - 1; L >= 0; --L) {
        const int32_t n = (int32_t)(c->solve_off[L + 1] - c->solve_off[L]);
        if ((e = launch_trsv_backward_level(nrhs, c->dSolveSn + c->solve_off[L], n, c->solve_maxfront[L], c->dSN,
                                            c->dL, c->dLinv, c->dRows, c->dXv, st)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

fetiF_status fetif::need_factors(fetiF_ctx c)
{
    if (c->n_uploaded != c->nsub) return fail(c, FETIF_ESTATE, "solve before every subdomain was factored");
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_apply_implicit(fetiF_ctx c, const double* lambda_d, double* q_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (!lambda_d || !q_d || lambda_d == q_d) return fail(c, FETIF_EINVAL, "lambda/q NULL or overlapping");
    if (fetiF_status st0 = need_factors(c)) return st0;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, order_after_upload(c, st));
    if (c->opt.debug_checks)
        if (fetiF_status s1 = debug_scan(c, 0, lambda_d, c->n_lambda, "fetiF_apply_implicit", "lambda", st)) return s1;
    {
        PhaseTimer t6(c, st, 6);
        HIPCHK(c, launch_scatter_dual(1, c->nsub, c->dSubRow, c->dSubM, c->dStartRows, c->dSignsSorted, c->dDmap,
                                      lambda_d, nullptr, c->dXv, c->total_rows, st));
        HIPCHK(c, solve_all(c, 1, st));
        HIPCHK(c, launch_xgather(1, c->n_lambda, c->dXGptr, c->dXGent, c->dXv, nullptr, q_d, st));
        HIPCHK(c, t6.stop());
    }
    if (c->opt.debug_checks) return debug_scan(c, 0, q_d, c->n_lambda, "fetiF_apply_implicit", "q", st);
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_dual_rhs(fetiF_ctx c, const double* f_d, const double* c_d, double* d_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (!f_d || !d_d) return fail(c, FETIF_EINVAL, "f or d is NULL");
    if (fetiF_status st0 = need_factors(c)) return st0;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, order_after_upload(c, st));
    PhaseTimer t6(c, st, 6);
    HIPCHK(c, launch_permute_in(c->total_rows, c->dXperm, f_d, c->dXv, st));
    HIPCHK(c, solve_all(c, 1, st));
    HIPCHK(c, launch_xgather(1, c->n_lambda, c->dXGptr, c->dXGent, c->dXv, c_d, d_d, st));
    HIPCHK(c, t6.stop());
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_apply_backward(fetiF_ctx c, const double* g_d, const double* lambda_d,
                                             double* dlambda_d, double* dtheta_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (!g_d || !dlambda_d || g_d == dlambda_d) return fail(c, FETIF_EINVAL, "g/dlambda NULL or overlapping");
    if (dtheta_d && !lambda_d) return fail(c, FETIF_EINVAL, "dtheta needs lambda");
    if (dtheta_d && !c->has_elems) return fail(c, FETIF_EINVAL, "dtheta needs element data at create");
    if (fetiF_status sa = apply_checks(c, g_d, dlambda_d)) return sa;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    const bool dbg = c->opt.debug_checks != 0;
    if (dbg) {
        if (fetiF_status s1 = debug_scan(c, 0, g_d, c->n_lambda, "fetiF_apply_backward", "g", st)) return s1;
        if (dtheta_d)
            if (fetiF_status s1 = debug_scan(c, 0, lambda_d, c->n_lambda, "fetiF_apply_backward", "lambda", st)) return s1;
    }
    // dlambda = F g (F~ is symmetric)
    fetiF_status st0 = apply_with_partials(c, g_d, dlambda_d, c->dZ, st);
    if (st0 != FETIF_OK) return st0;
    if (dbg)
        if (fetiF_status s1 = debug_scan(c, 0, dlambda_d, c->n_lambda, "fetiF_apply_backward", "dlambda", st)) return s1;
    if (!dtheta_d) return FETIF_OK;
    HIPCHK(c, order_after_upload(c, st));
    {
        PhaseTimer t6(c, st, 6);
        HIPCHK(c, launch_scatter_dual(2, c->nsub, c->dSubRow, c->dSubM, c->dStartRows, c->dSignsSorted, c->dDmap,
                                      g_d, lambda_d, c->dXv, c->total_rows, st));
        HIPCHK(c, solve_all(c, 2, st));
        HIPCHK(c, launch_elem_adjoint(c->nelem_total, c->dElems, c->dEpos, c->dDK, c->dXv, dtheta_d, st));
        HIPCHK(c, t6.stop());
    }
    if (dbg) return debug_scan(c, 0, dtheta_d, c->nelem_total, "fetiF_apply_backward", "dtheta", st);
    return FETIF_OK;
}

// ======================================================================== inspection

extern "C" fetiF_status fetiF_download_F(fetiF_ctx c, int32_t sub, double* host_out)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (sub < 0 || sub >= c->nsub || !host_out) return fail(c, FETIF_EINVAL, "bad subdomain or output");
    if (!c->assembled) return fail(c, FETIF_ESTATE, "download before assemble");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    const SubPlan& P = c->subs[sub];
    const int V = prec_row_align(c->prec), B = prec_bytes(c->prec);
    const int64_t fel = packed_row_offset(P.m, V);
    std::vector<char> buf((size_t)fel * B + 16);
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(buf.data(), (char*)c->dF + (size_t)P.fbase * B, (size_t)fel * B, hipMemcpyDeviceToHost));
    auto val = [&](int64_t e) -> double {
        if (c->prec == 0) {
            double v;
            std::memcpy(&v, buf.data() + e * 8, 8);
            return v;
        }
        if (c->prec == 1) {
            float v;
            std::memcpy(&v, buf.data() + e * 4, 4);
            return v;
        }
        uint16_t h;
        std::memcpy(&h, buf.data() + e * 2, 2);
        uint32_t u = (uint32_t)h << 16;
        float v;
        std::memcpy(&v, &u, 4);
        return v;
    };
    const int32_t m = P.m;
    for (int32_t a = 0; a < m; ++a) {
        const int64_t ro = packed_row_offset(a, V);
        for (int32_t b = 0; b <= a; ++b) {
            double v = val(ro + b);
            int32_t i = P.sigma[a], j = P.sigma[b];
            host_out[(size_t)i * m + j] = v;
            host_out[(size_t)j * m + i] = v;
        }
    }
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_query(fetiF_ctx c, fetiF_info* info)
{
    if (!c || !info) return FETIF_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->nsub = c->nsub;
    info->n_lambda = c->n_lambda;
    info->sum_m = c->sum_m;
    info->factor_values = c->total_L;
    info->x_values = c->total_X;
    info->f_elements = c->total_F;
    int64_t tri = 0;
    for (const auto& P : c->subs) tri += (int64_t)P.m * (P.m + 1) / 2;
    info->f_tri_elements = tri;
    info->trsm_flops = c->trsm_flops;
    info->syrk_flops = c->syrk_flops;
    info->factor_flops = c->factor_flops;
    info->trsm_levels = c->trsm_levels;
    info->trsm_bwd_flops = c->trsm_bwd_flops;
    info->apply_groups = c->ngroups;
    info->assembly_groups = (int32_t)c->grp_first.size() - 1;
    {
        const int V = prec_row_align(c->prec);
        int64_t tot = 0;
        for (const auto& P : c->subs) tot += packed_row_offset(P.m, V);
        info->apply_elements = tot;
    }
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_profile_enable(fetiF_ctx c, int on)
{
    if (!c) return FETIF_EINVAL;
    c->profiling = on != 0;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_profile_read(fetiF_ctx c, int reset, double* ms, int64_t* counts, int32_t nphases)
{
    if (!c) return FETIF_EINVAL;
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    for (auto& r : c->recs) {
        HIPCHK(c, hipEventSynchronize(r.b));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, r.a, r.b));
        c->prof_ms[r.phase] += t;
        c->prof_cnt[r.phase] += 1;
        c->ev_pool.push_back(r.a);
        c->ev_pool.push_back(r.b);
    }
    c->recs.clear();
    for (int32_t p = 0; p < nphases && p < FETIF_NPHASES; ++p) {
        if (ms) ms[p] = c->prof_ms[p];
        if (counts) counts[p] = c->prof_cnt[p];
    }
    if (reset)
        for (int p = 0; p < FETIF_NPHASES; ++p) {
            c->prof_ms[p] = 0.0;
            c->prof_cnt[p] = 0;
        }
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_destroy(fetiF_ctx c)
{
    if (!c) return FETIF_EINVAL;
    {
        DeviceGuard dg(c->device);
        (void)hipDeviceSynchronize();
        for (auto& r : c->recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
        if (c->pcpg_graph) (void)hipGraphExecDestroy(c->pcpg_graph);
        if (c->hHist) (void)hipHostFree(c->hHist);
        if (c->dHist) (void)hipFree(c->dHist);
        for (void* p : c->allocations) (void)hipFree(p);
        free_apply(c);
        free_trsm(c);
        free_bwd(c);
        if (c->dHostVec) (void)hipFree(c->dHostVec);
        if (c->dDmapId) (void)hipFree(c->dDmapId);
        if (c->hPin) (void)hipHostFree(c->hPin);
        if (c->hStage) (void)hipHostFree(c->hStage);
        if (c->hLbKval) (void)hipHostFree(c->hLbKval);
        if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    }
    delete c;
    return FETIF_OK;
}

extern "C" const char* fetiF_last_error(fetiF_ctx c)
{
    return c ? c->last_error.c_str() : g_create_error.c_str();
}
