// Host-only entry points: analysis and factorisation of one K_reg.
#include <cstring>
#include <new>
#include <string>

#include "../../include/fetiF.h"
#include "host_sparse.hpp"
#include "internal.hpp"

struct fetiF_hfactor_s {
    fetif::Symbolic sym;
    std::vector<double> panels;
};

namespace fetif {

bool pattern_from_sub(const fetiF_subdomain& s, Pattern& A, std::string& err)
{
    if (s.n <= 0 || !s.k_ptr || !s.k_idx) {
        err = "subdomain needs n > 0 and a CSR pattern";
        return false;
    }
    if (s.dofs_per_node <= 0 || s.n % s.dofs_per_node) {
        err = "n must be a multiple of dofs_per_node";
        return false;
    }
    A.n = s.n;
    A.ptr.assign(s.k_ptr, s.k_ptr + s.n + 1);
    if (A.ptr[0] != 0) {
        err = "k_ptr[0] must be 0";
        return false;
    }
    for (int32_t r = 0; r < s.n; ++r)
        if (A.ptr[r + 1] < A.ptr[r]) {
            err = "k_ptr not monotone";
            return false;
        }
    A.idx.assign(s.k_idx, s.k_idx + A.ptr[s.n]);
    return true;
}

bool multiplier_nodes(const fetiF_subdomain& s, std::vector<char>& flags)
{
    if (s.dofs_per_node <= 0 || s.n % s.dofs_per_node) return false;
    flags.assign((size_t)(s.n / s.dofs_per_node), 0);
    for (int32_t j = 0; j < s.m; ++j) {
        if (!s.b_dof || s.b_dof[j] < 0 || s.b_dof[j] >= s.n) return false;
        flags[(size_t)(s.b_dof[j] / s.dofs_per_node)] = 1;
    }
    return true;
}

void options_defaults(const fetiF_options* in, fetiF_options& o)
{
    std::memset(&o, 0, sizeof(o));
    if (in) o = *in;
    if (o.leaf_nodes <= 0) o.leaf_nodes = 24;
    if (o.apply_band <= 0) o.apply_band = 131072;
    if (o.trsm_chunk <= 0) o.trsm_chunk = 64;
    if (o.apply_rows != 2 && o.apply_rows != 4) o.apply_rows = 4;
    if (o.apply_nontemporal < 0 || o.apply_nontemporal > 1) o.apply_nontemporal = 1;
    if (o.apply_split < 0 || o.apply_split > 1) o.apply_split = 0;
    if (o.apply_seg != 0 && o.apply_seg != 2 && o.apply_seg != 3 && o.apply_seg != 4 && o.apply_seg != 8)
        o.apply_seg = 4;
    if (o.trsm_panel <= 0) o.trsm_panel = 48;
    o.trsm_panel = std::max(16, std::min(96, (o.trsm_panel + 15) / 16 * 16));
    if (o.assembly_groups <= 0) o.assembly_groups = 1;
    o.schur_order = o.schur_order != 0 ? 1 : 0;
    o.debug_checks = o.debug_checks != 0 ? 1 : 0;
}

}  // namespace fetif

using namespace fetif;

extern "C" fetiF_status fetiF_host_factor(const fetiF_subdomain* sub, const double* k_vals,
                                          const fetiF_options* opt, fetiF_hfactor* out)
{
    if (!sub || !out) return FETIF_EINVAL;
    *out = nullptr;
    fetiF_options o;
    options_defaults(opt, o);
    Pattern A;
    std::string err;
    if (!pattern_from_sub(*sub, A, err)) return FETIF_EINVAL;
    fetiF_hfactor_s* h = new (std::nothrow) fetiF_hfactor_s();
    if (!h) return FETIF_ENOMEM;
    SymbolicOptions so;
    so.leaf_nodes = o.leaf_nodes;
    std::vector<char> last;
    if (o.schur_order) {
        if (!multiplier_nodes(*sub, last)) {
            delete h;
            return FETIF_EINVAL;
        }
        so.last_nodes = &last;
    }
    int dim = sub->coords ? sub->dim : 0;
    if (!symbolic_analysis(A, sub->dofs_per_node, dim > 0 ? sub->coords : nullptr, dim, so, h->sym, err)) {
        delete h;
        return FETIF_EINVAL;
    }
    if (k_vals) {
        h->panels.assign((size_t)h->sym.nvals, 0.0);
        if (numeric_cholesky(h->sym, k_vals, h->panels.data()) >= 0) {
            delete h;
            return FETIF_ENOTSPD;
        }
    }
    *out = h;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_hfactor_info(fetiF_hfactor h, int32_t* n, int64_t* nnz, int32_t* nsuper,
                                           int32_t* nlevels)
{
    if (!h) return FETIF_EINVAL;
    int64_t z = 0;
    for (const auto& s : h->sym.sn) z += (int64_t)s.ncols * (s.ncols + 1) / 2 + (int64_t)s.ncols * s.nrows;
    if (n) *n = h->sym.n;
    if (nnz) *nnz = z;
    if (nsuper) *nsuper = (int32_t)h->sym.sn.size();
    if (nlevels) *nlevels = h->sym.nlevels;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_hfactor_export(fetiF_hfactor h, int32_t* perm, int64_t* colptr,
                                             int32_t* rowidx, double* vals)
{
    if (!h) return FETIF_EINVAL;
    const Symbolic& S = h->sym;
    if (perm) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * (size_t)S.n);
    int64_t p = 0;
    if (colptr) colptr[0] = 0;
    for (const auto& s : S.sn) {
        const int32_t d = s.ncols + s.nrows;
        for (int32_t k = 0; k < s.ncols; ++k) {
            for (int32_t i = k; i < d; ++i) {
                int32_t row = i < s.ncols ? s.first + i : S.rows[s.row_off + (i - s.ncols)];
                if (rowidx) rowidx[p] = row;
                if (vals) vals[p] = h->panels.empty() ? 0.0 : h->panels[s.val_off + (size_t)k * d + i];
                ++p;
            }
            if (colptr) colptr[s.first + k + 1] = p;
        }
    }
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_hfactor_supernodes(fetiF_hfactor h, int32_t* first, int32_t* ncols,
                                                 int32_t* nrows, int32_t* parent, int32_t* level)
{
    if (!h) return FETIF_EINVAL;
    const auto& sn = h->sym.sn;
    for (size_t s = 0; s < sn.size(); ++s) {
        if (first) first[s] = sn[s].first;
        if (ncols) ncols[s] = sn[s].ncols;
        if (nrows) nrows[s] = sn[s].nrows;
        if (parent) parent[s] = sn[s].parent;
        if (level) level[s] = sn[s].level;
    }
    return FETIF_OK;
}

extern "C" void fetiF_hfactor_free(fetiF_hfactor h) { delete h; }
