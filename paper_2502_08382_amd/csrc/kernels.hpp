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
                             const DevSN* sns, const double* L, const double* Linv, const int32_t* rows,
                             const XRow* xrows, double* X, hipStream_t st);
// dynamic LDS bytes of a TRSM level launch
inline size_t trsm_lds_bytes(int32_t waves, int32_t max_ns) { return (size_t)waves * ((max_ns + 15) / 16) * 2048; }
// prec: 0 f64, 1 f32, 2 bf16
hipError_t launch_syrk(int prec, const SyrkTile* tiles, int32_t ntiles, const int32_t* lists,
                       const DevSN* sns, const double* X, void* F, hipStream_t st);
// rows: rows per wavefront pass (1 or 2); ntl: non-temporal loads of F
hipError_t launch_apply_band(int prec, int nch, int rows, bool ntl, const Band* bands, int32_t nbands,
                             const void* F, const double* lam, const int32_t* dmap, void* z, hipStream_t st);
hipError_t launch_gather(int prec, int64_t n_lambda, const int32_t* gptr, const GatherEnt* ents,
                         const int64_t* band_zoff, const void* z, double* q, hipStream_t st);

// elements per 16-byte vector for a storage precision
inline int prec_vec(int prec) { return prec == 0 ? 2 : (prec == 1 ? 4 : 8); }
inline int prec_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

}  // namespace fetif
