// Host-side sparse direct-solver pieces that feed the device path:
// nested-dissection ordering, supernodal symbolic analysis and the numeric
// supernodal Cholesky K_reg = L L^T (paper Sec. III: symbolic stage once,
// numeric stage every step).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace fetif {

// Symmetric sparsity pattern, full (both triangles), CSR, sorted columns.
struct Pattern {
    int32_t n = 0;
    std::vector<int32_t> ptr;  // n+1
    std::vector<int32_t> idx;
};

// Fill-reducing order (new -> old) by nested dissection.  With node
// coordinates (nnodes x dim, row-major) the separators are coordinate
// planes through the median of the longest bounding-box axis, completed to a
// vertex separator of the graph; without coordinates the separator is the
// middle level of a breadth-first level structure.  DOFs of one node
// (dof = dpn*node + comp) stay together.
// With `last` (one flag per node), the flagged nodes are left out of the
// dissection and ordered after all others, ascending.
std::vector<int32_t> nested_dissection(const Pattern& A, int dpn, const double* coords, int dim,
                                       int leaf_nodes, const std::vector<char>* last = nullptr);

struct Supernode {
    int32_t first = 0;   // first column (permuted order)
    int32_t ncols = 0;
    int32_t nrows = 0;   // rows below the diagonal block
    int64_t row_off = 0; // offset into Symbolic::rows
    int64_t val_off = 0; // offset of the (ncols+nrows) x ncols column-major panel
    int32_t parent = -1; // supernode index, -1 for a root
    int32_t level = 0;   // height: 0 for leaves
};

// Supernodal structure of L for P K_reg P^T in postorder.
struct Symbolic {
    int32_t n = 0;
    std::vector<int32_t> perm;       // new -> old
    std::vector<int32_t> pinv;       // old -> new
    std::vector<Supernode> sn;
    std::vector<int32_t> rows;       // per supernode: its below-diagonal rows (ascending)
    std::vector<int32_t> col2sn;     // column -> supernode
    int64_t nvals = 0;               // total panel entries
    int32_t nlevels = 0;
    // permuted lower-triangle of A for the numeric phase: for each column j,
    // entries (row >= j, position in the caller's CSR value array)
    std::vector<int32_t> acol_ptr;   // n+1
    std::vector<int32_t> acol_row;
    std::vector<int32_t> acol_src;
    double flops_factor = 0.0;
};

struct SymbolicOptions {
    int leaf_nodes = 24;
    // relaxed amalgamation: merge a child supernode into its parent when the
    // merged supernode has at most relax_cols[k] columns and the fraction of
    // explicit zeros stays below relax_zeros[k-1] (any zeros for k=0).  The
    // caps keep large separators apart: merging them would widen the RHS
    // column range of the smaller one in the sparse-RHS triangular solve.
    int relax_cols[4] = {4, 16, 48, 96};
    double relax_zeros[3] = {0.8, 0.2, 0.05};
    // nodes ordered last (one flag per node), or none: the Schur-complement
    // route orders the nodes that carry Lagrange multipliers last, so the
    // trailing block of L is the Cholesky factor of the Schur complement of
    // the interior and the RHS columns of B~^T start in it
    const std::vector<char>* last_nodes = nullptr;
};

bool symbolic_analysis(const Pattern& A, int dpn, const double* coords, int dim,
                       const SymbolicOptions& opt, Symbolic& out, std::string& err);

// Numeric supernodal Cholesky (multifrontal, dense fronts).  vals are the
// caller's CSR values (same pattern as given to symbolic_analysis); panels
// receives sym.nvals doubles.  Returns -1 on success, else the permuted
// column whose pivot was not positive.
int32_t numeric_cholesky(const Symbolic& sym, const double* vals, double* panels);

}  // namespace fetif
