// Launchers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "device_types.hpp"

namespace fetif {

struct RhsUnit {
    int64_t off;   // element of X holding the unit entry of one RHS column
    double sign;   // +1 or -1
};

hipError_t launch_fill_zero(double* x, int64_t n, hipStream_t st);
hipError_t launch_rhs_units(const RhsUnit* u, int64_t n, double* X, hipStream_t st);
// inverses of the 16x16 diagonal blocks of the supernode panels
hipError_t launch_diag_inverse(const InvItem* items, int32_t nitems, const DevSN* sns, const double* L,
                               double* Linv, hipStream_t st);
// one etree level of the supernodal forward solve; waves = wavefronts per
// work-group (each owns 16 RHS columns), max_ns = largest supernode of the level
hipError_t launch_trsm_level(const TrsmItem* items, int32_t nitems, int32_t waves, int32_t max_ns,
                             const DevSN* sns, const double* L, const double* Linv, const int64_t* rowoff,
                             double* X, hipStream_t st);
// TRSM path (two TRSMs + SpMM): one level of the backward solve Z = L^{-T} X
// over column panels of every supernode (dense RHS, all m_i columns;
// pans[].pad = m_i, zrow = Z offsets of each panel's rows then below rows)
hipError_t launch_trsm_bwd_level(const TrsmItem* items, int32_t nitems, int32_t waves, const DevSN* pans,
                                 const double* L, const double* Linv, const int64_t* zrow, const double* X, double* Z,
                                 hipStream_t st);
// F~_i = B~_i P^T Z_i into the packed triangles (nrows = sum m_i)
hipError_t launch_tri_from_z(int prec, int32_t nsub, int64_t nrows, const int32_t* sub_m, const int32_t* start_rows,
                             const int8_t* signs, const int64_t* zbase, const int64_t* fbase, const double* Z,
                             void* F, hipStream_t st);
// dynamic LDS bytes of a TRSM level launch
inline size_t trsm_lds_bytes(int32_t waves, int32_t max_ns) { return (size_t)waves * ((max_ns + 15) / 16) * 2048; }
// ---- batched supernodal solves with L (nrhs = 1 or 2, vectors interleaved:
// x[row * nrhs + r]); x holds the right-hand side on entry, the solution on exit
// scatter: x_i = P_i B~_i^T D_i v (for each rhs vector v_r), x zeroed first
hipError_t launch_scatter_dual(int nrhs, int32_t nsub, const int32_t* sub_rowbase, const int32_t* sub_mbase,
                               const int32_t* start_rows, const int8_t* signs_sorted, const int32_t* dmap_sorted,
                               const double* v0, const double* v1, double* x, int64_t nrows_total,
                               hipStream_t st);
hipError_t launch_trsv_forward_level(int nrhs, const int32_t* sn_list, int32_t n, int32_t max_front,
                                     const DevSN* sns, const double* L, const double* Linv,
                                     const int32_t* child_ptr, const int32_t* child_idx, const int32_t* relpos,
                                     double* u, double* x, hipStream_t st);
hipError_t launch_trsv_backward_level(int nrhs, const int32_t* sn_list, int32_t n, int32_t max_front,
                                      const DevSN* sns, const double* L, const double* Linv, const int32_t* rows,
                                      double* x, hipStream_t st);
// q[g] = sum of sign * x[xpos] over the entries of g (rhs slot 0 of an nrhs
// layout), minus c[g] when c is not NULL
hipError_t launch_xgather(int nrhs, int64_t n_lambda, const int32_t* gptr, const XGatherEnt* ents, const double* x,
                          const double* c, double* q, hipStream_t st);
// x[r] = f[xperm[r]] (one rhs)
hipError_t launch_permute_in(int64_t n, const int32_t* xperm, const double* f, double* x, hipStream_t st);
// dtheta_e = -x0|_e^T dK x1|_e (slots 0 and 1 of a 2-rhs layout)
hipError_t launch_elem_adjoint(int64_t nelem, const ElemRef* elems, const int32_t* epos, const double* dk,
                               const double* x, double* dtheta, hipStream_t st);

// prec: 0 f64, 1 f32, 2 bf16
hipError_t launch_syrk(int prec, const SyrkTile* tiles, int32_t ntiles, const int32_t* lists,
                       const DevSN* sns, const double* X, void* F, hipStream_t st);
// rows: rows per pass of a wavefront pair (2 or 4); ntl: non-temporal loads
// of F; work-group g handles the segments bands[seg_ptr[g] .. seg_ptr[g+1])
hipError_t launch_apply_band(int prec, int nch, int rows, bool ntl, const Band* bands, const int32_t* seg_ptr,
                             int32_t ngroups, const void* F, const double* lam, const int32_t* dmap, void* z,
                             hipStream_t st);
// column-segmented apply: segch chunks per segment (4 or 8); brmax = most
// rows of a band (1 .. kMaxBandRows); any m
hipError_t launch_apply_seg(int prec, int segch, int rows, bool ntl, const Band* bands, const int32_t* seg_ptr,
                            int32_t ngroups, const void* F, const double* lam, const int32_t* dmap, void* z,
                            int32_t brmax, hipStream_t st);
// most rows of one apply band: the segmented kernel keeps p and the row
// sums of a band's rows in LDS (with FP64 partials and 8-chunk segments,
// 2 * 8 * 3072 + 2 * 8 * 1024 bytes = 64 KiB)
constexpr int32_t kMaxBandRows = 3072;
// columns the whole-row kernel can hold (its LDS keeps p for all of them)
constexpr int32_t kMaxWholeRowCols = 4096;
// dynamic LDS of the segmented kernel: p and the sums of the segment's
// columns and of the band's rows, in the accumulation type
inline size_t apply_seg_lds_bytes(int prec, int segch, int32_t brmax)
{
    const size_t acc = prec == 0 ? 8 : 4;
    const size_t segw = (size_t)segch * 64 * (16 / (prec == 0 ? 8 : (prec == 1 ? 4 : 2)));
    return acc * (2 * segw + 2 * (size_t)brmax);
}
// q[g] = sum of z[zpos[k]] for k in [zptr[g], zptr[g+1]), in that order
hipError_t launch_gather(int prec, int64_t n_lambda, const int32_t* zptr, const int64_t* zpos, const void* z,
                         double* q, hipStream_t st);

// streaming-read probe: work-group g sums bytes [g region, (g+1) region) of
// buf as FP64 values into out[g] (ceil(bytes / region) work-groups)
hipError_t launch_read_probe(const void* buf, int64_t bytes, int64_t region, double* out, hipStream_t st);

// Size of the file-scope device array `scratch` (kernels.hip) that holds the
// apply partial vectors of the allocation-free apply: one copy per device,
// held until the process ends.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Device address of `scratch` on `device`, which must be the current device:
// looked up with hipGetSymbolAddress on the first call per device and cached.
hipError_t static_scratch_address(int device, void** out);

// elements per 16-byte vector for a storage precision
inline int prec_vec(int prec) { return prec == 0 ? 2 : (prec == 1 ? 4 : 8); }
inline int prec_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
// row granularity of the packed triangles (elements per 128-byte line)
inline int prec_row_align(int prec) { return kRowAlignBytes / prec_bytes(prec); }

}  // namespace fetif
