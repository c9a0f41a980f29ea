// Plain-old-data records shared by the host planner and the HIP kernels.
#pragma once
#include <cstdint>

namespace fetif {

// One supernode of one subdomain, in device form.  The TRSM also uses
// records of column panels of a supernode (a view of the same storage at
// diagonal offset o: ncols <= the panel width, the supernode's later columns
// counted among its below rows, ld the supernode's leading dimension).
struct DevSN {
    int64_t lval;    // offset of its column-major panel (ncols columns, ld rows) in the factor buffer
    int64_t linv;    // offset of the inverses of its 16x16 diagonal blocks (-1: none)
    int64_t xoff;    // offset of its ncols x w row-major block of X
    int64_t rowsoff; // offset of its below-diagonal row list (subdomain-local rows)
    int32_t rowbase; // first global row slot of its subdomain (for the X row tables)
    int32_t first;   // first column (subdomain-local, permuted order)
    int32_t ncols;
    int32_t nrows;
    int32_t j0;      // first RHS column of its range (sorted local multiplier order)
    int32_t w;       // width of its RHS column range
    int32_t ld;      // leading dimension of the panel (ncols + nrows for a whole supernode)
    int32_t pad;
};

// Diagonal-block inversion item: block rb of supernode sn.
struct InvItem {
    int32_t sn;
    int32_t rb;
};

// TRSM work item: one RHS column chunk of one supernode.
struct TrsmItem {
    int32_t sn;      // global supernode index
    int32_t c0;      // first column of the chunk, relative to j0
    int32_t cw;      // chunk width
    int32_t pad;
};

// X row table: row r of subdomain i lives at X[off + (j - j0)] for RHS
// columns j in [j0, j0 + w) of its supernode.
struct XRow {
    int64_t off;
    int32_t j0;
    int32_t w;
};

// SYRK output tile: rows [ta*T, ..) x cols [tb*T, ..) of F~_i (sorted order).
struct SyrkTile {
    int64_t fbase;   // element offset of F~_i in the F buffer
    int32_t m;       // size of F~_i
    int32_t ta, tb;  // tile coordinates, ta >= tb
    int32_t list0;   // contributing supernodes: syrk_list[list0 .. list1)
    int32_t list1;
    int32_t pad;
};

// Apply work unit: rows [r0, r1) of the packed lower triangle of F~_i.
struct Band {
    int64_t fbase;   // element offset of F~_i
    int64_t zoff;    // offset of the band's partial vector (length r1)
    int32_t r0, r1;
    int32_t dbase;   // offset of D_i (sorted order) in the dual-map buffer
    int32_t pad;
};

// Implicit-apply gather entry: one (subdomain, local multiplier) term of a
// global multiplier, read from the solved vector at `xpos` with `sign`.
struct XGatherEnt {
    int64_t xpos;
    double sign;
};

// Element of the theta-adjoint: its subdomain and the offset of its
// permuted DOF positions (edofs entries) in the element-position table.
struct ElemRef {
    int32_t sub;
    int32_t edofs;
    int64_t pos_off;  // into the element-position table (global x rows)
    int64_t dk_off;   // into the dK table (edofs x edofs, row-major)
};

// Rows of a packed triangle F~_i start on 128-byte boundaries (the cache
// line): no line holds parts of two rows, so work split by rows or by
// 1 KiB chunks of a row never fetches a line twice.
constexpr int kRowAlignBytes = 128;

// Packed lower-triangle row offset with rows padded to multiples of V
// elements: row r holds columns 0..r and starts at
// V * (V*q*(q+1)/2 + s*(q+1)) where r = q*V + s.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline int64_t packed_row_offset(int64_t r, int64_t V)
{
    int64_t q = r / V, s = r - q * V;
    return V * (V * q * (q + 1) / 2 + s * (q + 1));
}

}  // namespace fetif
