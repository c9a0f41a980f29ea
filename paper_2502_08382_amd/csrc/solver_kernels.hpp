// Records and launchers of the solver kernels (solver.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace fetif {

constexpr int COARSE_MAXK = 6;  // kernel dimension per subdomain (3D elasticity: 6)
// The deterministic dots use up to 64 work-groups of 256 threads
// (grid-stride beyond), so their partial count depends on n only; the
// partial buffer holds 2 * dot_parts(n_lambda) values.  More work-groups
// measured slower: every one of them adds an atomic on the completion
// counter and a partial to the last work-group's sum (256 instead of 64:
// about 2 us more per dot at 221,600 multipliers).
inline int32_t dot_parts(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int32_t)(b < 1 ? 1 : (b > 64 ? 64 : b));
}

// solver scalars in device memory
enum { SC_WY = 0, SC_PQ, SC_DELTA, SC_BETA, SC_WW, SC_TMP, SC_TMP2, SC_K, SC_COUNT };

// coarse-space block of one subdomain: G_i = D_i^T B~_i R_i
struct CoarseSub {
    int64_t mbase;   // first sorted local multiplier (into the sorted dual map)
    int64_t gvbase;  // first value of its G rows (m x nk, sorted multiplier order)
    int64_t rbase;   // first row of R_i in the concatenated R (n rows of nk)
    int32_t m;
    int32_t nk;
    int32_t koff;    // first coarse unknown (alpha index)
    int32_t n;
    int32_t rowbase; // first entry of the subdomain in the concatenated DOF vector
    int32_t pad;
};

// one term of row g of G: Gv[gv .. gv+nk) against s[koff .. koff+nk)
struct GEnt {
    int64_t gv;
    int32_t koff;
    int32_t nk;
};

hipError_t launch_gt(int32_t nsub, const CoarseSub* cs, const double* gv, const int32_t* dmap, const double* w,
                     double* t, hipStream_t st);
hipError_t launch_rtf(int32_t nsub, const CoarseSub* cs, const double* R, const double* f, double* e, hipStream_t st);
hipError_t launch_gemv(int32_t nc, const double* A, const double* x, double* y, hipStream_t st);
hipError_t launch_gs(int64_t n, double alpha, double sgn, const int32_t* gptr, const GEnt* ents, const double* gv,
                     const double* s, const double* w, double* out, hipStream_t st);
// deterministic dot(s) x.y (and x.z if z) followed by the scalar update
// `mode`; the history index is a device counter (graph-replay safe)
hipError_t launch_dot(int64_t n, const double* x, const double* y, const double* z, int mode, double* part,
                      double* sc, double* hist, int32_t hist_cap, hipStream_t st);
hipError_t launch_update_lr(int64_t n, const double* sc, const double* p, const double* q, double* lam, double* r,
                            hipStream_t st);
hipError_t launch_update_p(int64_t n, int use_beta, const double* sc, const double* y, double* p, hipStream_t st);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                        hipStream_t st);
// Lumped preconditioner y = sum_i D_i^T B~_i K_reg,i B~_i^T D_i w (the M of
// Alg. 1).  Per subdomain: its first boundary-DOF slot (global), count, and
// first sorted multiplier position.
struct LumpSub {
    int32_t bbase, nb, dbase, m;
};
// ylocal[dbase + k] = sign_k (K_bb x)[b_k] with x = B~^T D w on the boundary
// DOFs; one work-group per subdomain, 2 * nbmax doubles of LDS
hipError_t launch_lumped_local(int32_t nsub, int32_t nbmax, const LumpSub* ls, const int32_t* uptr,
                               const int32_t* uk, const double* sgn, const int32_t* kptr, const int32_t* kcol,
                               const double* kval, const int32_t* mb, const int32_t* dmap, const double* w,
                               double* ylocal, hipStream_t st);
// y = A^{-1} x with the dense inverses of the diagonal blocks of A (the
// scaled jump operator's B W B^T): block sb_of[g], members sb_mem[sb_ptr[b] ..
// sb_ptr[b+1]), inverse (row-major) at sb_off[b]
hipError_t launch_block_apply(int64_t n, const int32_t* sb_of, const int32_t* sb_pos, const int32_t* sb_ptr,
                              const int32_t* sb_mem, const int64_t* sb_off, const double* inv, const double* x,
                              double* y, hipStream_t st);
// y[g] = sum of ylocal over the sorted positions of multiplier g (fixed order)
hipError_t launch_lumped_gather(int64_t n, const int32_t* gptr, const int32_t* gpos, const double* ylocal,
                                double* y, hipStream_t st);
hipError_t launch_gauss_jordan_inverse(int32_t n, double* A, double* rowk, double* colk, hipStream_t st);
hipError_t launch_permute_out(int64_t n, const int32_t* xperm, const double* x, double* u, hipStream_t st);
hipError_t launch_add_kernel_part(int32_t nsub, const CoarseSub* cs, const double* R, const double* alpha, double* u,
                                  hipStream_t st);
hipError_t launch_load_primal_rhs(int32_t nsub, const int32_t* sub_rowbase, const int32_t* sub_mbase,
                                  const int32_t* xperm, const int32_t* start_rows, const int8_t* signs,
                                  const int32_t* dmap, const double* f, const double* lam, double* x, hipStream_t st);


// Debug scan: first[0] = the index of the first element of x[0, n) that is
// NaN or Inf, all ones when there is none; elements of precision prec (0
// FP64, 1 FP32, 2 BF16 bits).
hipError_t launch_first_nonfinite(int prec, const void* x, int64_t n, unsigned long long* first, hipStream_t st);

}  // namespace fetif
