// Kernels of the projected conjugate gradient solver (paper Alg. 1) and of
// the coarse space G = B R, P = I - G (G^T G)^{-1} G^T (Sec. II).  FP64.
// Reductions use a fixed grid and a fixed tree, so results are bitwise
// reproducible; solver scalars live in device memory (no host round trip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "solver_kernels.hpp"

namespace fetif {

namespace {

constexpr int NT = 256;

// Sum over the work-group, returned to every thread: a butterfly inside each
// wavefront, then the wavefront sums added in wavefront order (a fixed tree,
// so the result does not depend on timing).  sh holds NT / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();  // an earlier call may still be reading sh
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) r += sh[k];
    return r;
}

// t[koff_i + k] = sum_j Gv[j][k] w[D_j] over the local multipliers j of
// subdomain i (one work-group per subdomain).
__global__ __launch_bounds__(NT) void gt_kernel(const CoarseSub* __restrict__ cs, const double* __restrict__ gv,
                                                const int32_t* __restrict__ dmap, const double* __restrict__ w,
                                                double* __restrict__ t)
{
    __shared__ double sh[NT / 64];
    const CoarseSub c = cs[blockIdx.x];
    double acc[COARSE_MAXK];
#pragma unroll
    for (int k = 0; k < COARSE_MAXK; ++k) acc[k] = 0.0;
    for (int j = threadIdx.x; j < c.m; j += NT) {
        const double wj = w[dmap[c.mbase + j]];
        const double* g = gv + c.gvbase + (int64_t)j * c.nk;
#pragma unroll
        for (int k = 0; k < COARSE_MAXK; ++k)
            if (k < c.nk) acc[k] += g[k] * wj;
    }
#pragma unroll
    for (int k = 0; k < COARSE_MAXK; ++k) {
        if (k >= c.nk) break;
        const double s = block_sum(acc[k], sh);
        if (threadIdx.x == 0) t[c.koff + k] = s;
    }
}

// y = A x for a dense nc x nc row-major A (one wavefront per row).
__global__ __launch_bounds__(NT) void gemv_kernel(int32_t nc, const double* __restrict__ A,
                                                  const double* __restrict__ x, double* __restrict__ y)
{
    const int row = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nc) return;
    const double* a = A + (int64_t)row * nc;
    double acc = 0.0;
    for (int k = lane; k < nc; k += 64) acc += a[k] * x[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) y[row] = acc;
}

// out[g] = alpha * w[g] + sgn * sum_{entries of g} Gv[e] . s[koff .. koff+nk)
__global__ __launch_bounds__(NT) void gs_kernel(int64_t n, double alpha, double sgn, const int32_t* __restrict__ gptr,
                                                const GEnt* __restrict__ ents, const double* __restrict__ gv,
                                                const double* __restrict__ s, const double* __restrict__ w,
                                                double* __restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n) return;
    double acc = 0.0;
    for (int32_t e = gptr[g]; e < gptr[g + 1]; ++e) {
        const GEnt E = ents[e];
        const double* v = gv + E.gv;
        for (int k = 0; k < E.nk; ++k) acc += v[k] * s[E.koff + k];
    }
    out[g] = (w ? alpha * w[g] : 0.0) + sgn * acc;
}

// Deterministic completion of up to two grid-wide sums (a, b): each
// work-group writes its partials; the last one to finish (counted with an
// atomic on `done`) adds the partials in a fixed order, updates the solver
// scalars and resets the counter (so a captured graph can be replayed
// without clearing anything).  Called by every thread of every work-group.
//  mode 0 (init):   wy = a, ww = b, k = 0, hist[0] = ww
//  mode 1 (delta):  pq = a, delta = wy / pq
//  mode 2 (beta):   beta = a / wy, wy = a, ww = b, k += 1, hist[k] = ww
//  mode 3 (plain):  sc[SC_TMP] = a, sc[SC_TMP2] = b
__device__ void finish_sums(double a, double b, int mode, double* __restrict__ part, double* __restrict__ sc,
                            double* __restrict__ hist, int32_t cap, unsigned int* done, double* sh)
{
    __shared__ bool last;
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
        __threadfence();
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const int nparts = (int)gridDim.x;
    a = 0.0;
    b = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) {
        a += __builtin_nontemporal_load(part + i);
        b += __builtin_nontemporal_load(part + nparts + i);
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x != 0) return;
    *done = 0u;
    if (mode == 0) {
        sc[SC_WY] = a;
        sc[SC_WW] = b;
        sc[SC_K] = 0.0;
        if (hist && cap > 0) hist[0] = b;
    } else if (mode == 1) {
        sc[SC_PQ] = a;
        sc[SC_DELTA] = a != 0.0 ? sc[SC_WY] / a : 0.0;
    } else if (mode == 2) {
        const double wy = sc[SC_WY];
        sc[SC_BETA] = wy != 0.0 ? a / wy : 0.0;
        sc[SC_WY] = a;
        sc[SC_WW] = b;
        const int k = (int)sc[SC_K] + 1;
        sc[SC_K] = (double)k;
        if (hist && k < cap) hist[k] = b;
    } else {
        sc[SC_TMP] = a;
        sc[SC_TMP2] = b;
    }
}

// x.y (and x.z when z != NULL) over dot_parts(n) work-groups, then the scalar
// update `mode` of finish_sums.  Each thread requests its (up to) four
// elements of a pass before adding them.
__global__ __launch_bounds__(NT) void dot_kernel(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ y, const double* __restrict__ z,
                                                 int mode, double* __restrict__ part, double* __restrict__ sc,
                                                 double* __restrict__ hist, int32_t cap, unsigned int* done)
{
    __shared__ double sh[NT / 64];
    const int64_t stride = (int64_t)gridDim.x * NT;
    double a = 0.0, b = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * NT + threadIdx.x; i0 < n; i0 += 4 * stride) {
        double xv[4], yv[4], zv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = i0 + k * stride;
            const bool in = i < n;
            xv[k] = in ? x[i] : 0.0;
            yv[k] = in ? y[i] : 0.0;
            zv[k] = in && z ? z[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a += xv[k] * yv[k];
            b += xv[k] * zv[k];
        }
    }
    finish_sums(a, b, mode, part, sc, hist, cap, done, sh);
}

// Lumped preconditioner, local part: one work-group per subdomain.  x lives
// on the subdomain's boundary DOFs (x_u = sum of coef_k w[D k] over the
// multipliers k on DOF u, in a fixed order), t = K_bb x row by row, and
// every multiplier k takes coef_k t[b_k].  coef is the sign of B~ (lumped
// M) or the sign times the weight of the scaled jump operator.  uk and mb
// hold global sorted multiplier positions / boundary slots; kcol global
// boundary slots.
__global__ __launch_bounds__(NT) void lumped_local_kernel(const LumpSub* __restrict__ ls,
                                                          const int32_t* __restrict__ uptr,
                                                          const int32_t* __restrict__ uk,
                                                          const double* __restrict__ sgn,
                                                          const int32_t* __restrict__ kptr,
                                                          const int32_t* __restrict__ kcol,
                                                          const double* __restrict__ kval,
                                                          const int32_t* __restrict__ mb,
                                                          const int32_t* __restrict__ dmap,
                                                          const double* __restrict__ w, double* __restrict__ ylocal,
                                                          int32_t nbmax)
{
    extern __shared__ double lsm[];
    double* __restrict__ x = lsm;
    double* __restrict__ t = lsm + nbmax;
    const LumpSub S = ls[blockIdx.x];
    for (int u = threadIdx.x; u < S.nb; u += NT) {
        const int32_t g = S.bbase + u;
        double a = 0.0;
        for (int32_t e = uptr[g]; e < uptr[g + 1]; ++e) a += sgn[uk[e]] * w[dmap[uk[e]]];
        x[u] = a;
    }
    __syncthreads();
    for (int u = threadIdx.x; u < S.nb; u += NT) {
        const int32_t g = S.bbase + u;
        double a = 0.0;
        for (int32_t e = kptr[g]; e < kptr[g + 1]; ++e) a += kval[e] * x[kcol[e] - S.bbase];
        t[u] = a;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < S.m; k += NT) {
        const int32_t p = S.dbase + k;
        ylocal[p] = sgn[p] * t[mb[p] - S.bbase];
    }
}

// y = A^{-1} x for the block-diagonal A of the scaled jump operator: every
// multiplier g takes the row of its block's dense inverse times the block's
// entries of x (one thread per multiplier; blocks hold a handful of
// multipliers: those sharing a DOF of some subdomain).
__global__ __launch_bounds__(NT) void block_apply_kernel(int64_t n, const int32_t* __restrict__ sb_of,
                                                         const int32_t* __restrict__ sb_pos,
                                                         const int32_t* __restrict__ sb_ptr,
                                                         const int32_t* __restrict__ sb_mem,
                                                         const int64_t* __restrict__ sb_off,
                                                         const double* __restrict__ inv,
                                                         const double* __restrict__ x, double* __restrict__ y)
{
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n) return;
    const int32_t b = sb_of[g];
    const int32_t p0 = sb_ptr[b], s = sb_ptr[b + 1] - p0;
    const double* __restrict__ row = inv + sb_off[b] + (int64_t)sb_pos[g] * s;
    double a = 0.0;
    for (int32_t j = 0; j < s; ++j) a += row[j] * x[sb_mem[p0 + j]];
    y[g] = a;
}

__global__ __launch_bounds__(NT) void lumped_gather_kernel(int64_t n, const int32_t* __restrict__ gptr,
                                                           const int32_t* __restrict__ gpos,
                                                           const double* __restrict__ ylocal, double* __restrict__ y)
{
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n) return;
    double a = 0.0;
    for (int32_t e = gptr[g]; e < gptr[g + 1]; ++e) a += ylocal[gpos[e]];
    y[g] = a;
}

// lambda += delta p ; r -= delta q
__global__ __launch_bounds__(NT) void update_lr_kernel(int64_t n, const double* __restrict__ sc,
                                                       const double* __restrict__ p, const double* __restrict__ q,
                                                       double* __restrict__ lam, double* __restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const double d = sc[SC_DELTA];
    lam[i] += d * p[i];
    r[i] -= d * q[i];
}

// p = y + beta p (beta from the scalars; use_beta = 0 gives p = y)
__global__ __launch_bounds__(NT) void update_p_kernel(int64_t n, int use_beta, const double* __restrict__ sc,
                                                      const double* __restrict__ y, double* __restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    p[i] = use_beta ? y[i] + sc[SC_BETA] * p[i] : y[i];
}

// out = a x + b y
__global__ __launch_bounds__(NT) void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                                                   const double* __restrict__ y, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) out[i] = a * x[i] + b * y[i];
}

// Gauss-Jordan step k on an SPD matrix (in place, no pivoting): the row and
// column of the pivot are copied first so every element reads old values.
__global__ __launch_bounds__(NT) void gj_copy_kernel(int32_t n, int32_t k, const double* __restrict__ A,
                                                     double* __restrict__ rowk, double* __restrict__ colk)
{
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i < n) {
        rowk[i] = A[(int64_t)k * n + i];
        colk[i] = A[(int64_t)i * n + k];
    }
}

__global__ __launch_bounds__(NT) void gj_update_kernel(int32_t n, int32_t k, double* __restrict__ A,
                                                       const double* __restrict__ rowk,
                                                       const double* __restrict__ colk)
{
    const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
    const double inv = 1.0 / rowk[k];
    double v;
    if (i == k && j == k) v = inv;
    else if (i == k) v = rowk[j] * inv;
    else if (j == k) v = -colk[i] * inv;
    else v = A[idx] - colk[i] * rowk[j] * inv;
    A[idx] = v;
}

// u[rowbase + perm[k]] = x[rowbase + k]  (permuted rows back to DOF order)
__global__ __launch_bounds__(NT) void permute_out_kernel(int64_t n, const int32_t* __restrict__ xperm,
                                                         const double* __restrict__ x, double* __restrict__ u)
{
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (r < n) u[xperm[r]] = x[r];
}

// u[dof] += sum_k R_i[dof][k] alpha[koff_i + k]  (one work-group per subdomain)
__global__ __launch_bounds__(NT) void add_kernel_part(const CoarseSub* __restrict__ cs, const double* __restrict__ R,
                                                      const double* __restrict__ alpha, double* __restrict__ u)
{
    const CoarseSub c = cs[blockIdx.x];
    for (int r = threadIdx.x; r < c.n; r += NT) {
        const double* rr = R + (c.rbase + (int64_t)r) * c.nk;
        double acc = 0.0;
        for (int k = 0; k < c.nk; ++k) acc += rr[k] * alpha[c.koff + k];
        u[c.rowbase + r] += acc;
    }
}

// x_perm = P (f - B~^T D lambda) for one subdomain per work-group, with the
// local multipliers sorted by their permuted DOF (runs summed in order).
__global__ __launch_bounds__(NT) void load_primal_rhs_kernel(const int32_t* __restrict__ sub_rowbase,
                                                             const int32_t* __restrict__ sub_mbase,
                                                             const int32_t* __restrict__ xperm,
                                                             const int32_t* __restrict__ start_rows,
                                                             const int8_t* __restrict__ signs,
                                                             const int32_t* __restrict__ dmap,
                                                             const double* __restrict__ f,
                                                             const double* __restrict__ lam, double* __restrict__ x)
{
    const int i = blockIdx.x;
    const int rb = sub_rowbase[i], r1 = sub_rowbase[i + 1];
    const int m0 = sub_mbase[i], m1 = sub_mbase[i + 1];
    for (int r = rb + threadIdx.x; r < r1; r += NT) x[r] = f[xperm[r]];
    __syncthreads();
    for (int a = m0 + threadIdx.x; a < m1; a += NT) {
        const int row = start_rows[a];
        if (a > m0 && start_rows[a - 1] == row) continue;
        double acc = 0.0;
        for (int b = a; b < m1 && start_rows[b] == row; ++b) acc += (double)signs[b] * lam[dmap[b]];
        x[rb + row] -= acc;
    }
}

// e[koff_i + k] = sum_r R_i[r][k] f[rowbase_i + r]  (one work-group per subdomain)
__global__ __launch_bounds__(NT) void rtf_kernel(const CoarseSub* __restrict__ cs, const double* __restrict__ R,
                                                 const double* __restrict__ f, double* __restrict__ e)
{
    __shared__ double sh[NT / 64];
    const CoarseSub c = cs[blockIdx.x];
    double acc[COARSE_MAXK];
#pragma unroll
    for (int k = 0; k < COARSE_MAXK; ++k) acc[k] = 0.0;
    for (int r = threadIdx.x; r < c.n; r += NT) {
        const double fr = f[c.rowbase + r];
        const double* rr = R + (c.rbase + (int64_t)r) * c.nk;
#pragma unroll
        for (int k = 0; k < COARSE_MAXK; ++k)
            if (k < c.nk) acc[k] += rr[k] * fr;
    }
#pragma unroll
    for (int k = 0; k < COARSE_MAXK; ++k) {
        if (k >= c.nk) break;
        const double s = block_sum(acc[k], sh);
        if (threadIdx.x == 0) e[c.koff + k] = s;
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// Debug scan: the smallest index of a NaN or Inf among x[0, n) (an element
// is non-finite when its exponent bits are all ones), kept by a vector atomic
// minimum on first[0].
template <int BYTES>
__global__ __launch_bounds__(NT) void first_nonfinite_kernel(const void* __restrict__ x, int64_t n,
                                                             unsigned long long* __restrict__ first)
{
    unsigned long long mine = ~0ull;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        bool bad;
        if constexpr (BYTES == 8) bad = ((static_cast<const uint64_t*>(x)[i] >> 52) & 0x7ff) == 0x7ff;
        else if constexpr (BYTES == 4) bad = ((static_cast<const uint32_t*>(x)[i] >> 23) & 0xff) == 0xff;
        else bad = ((static_cast<const uint16_t*>(x)[i] >> 7) & 0xff) == 0xff;
        if (bad) {
            mine = (unsigned long long)i;
            break;
        }
    }
    if (mine != ~0ull) atomicMin(first, mine);
}

__global__ void set_all_ones_kernel(unsigned long long* p) { *p = ~0ull; }

}  // namespace

hipError_t launch_gt(int32_t nsub, const CoarseSub* cs, const double* gv, const int32_t* dmap, const double* w,
                     double* t, hipStream_t st)
{
    hipLaunchKernelGGL(gt_kernel, dim3(nsub), dim3(NT), 0, st, cs, gv, dmap, w, t);
    return hipGetLastError();
}

hipError_t launch_rtf(int32_t nsub, const CoarseSub* cs, const double* R, const double* f, double* e, hipStream_t st)
{
    hipLaunchKernelGGL(rtf_kernel, dim3(nsub), dim3(NT), 0, st, cs, R, f, e);
    return hipGetLastError();
}

hipError_t launch_gemv(int32_t nc, const double* A, const double* x, double* y, hipStream_t st)
{
    hipLaunchKernelGGL(gemv_kernel, dim3((unsigned)((nc + 3) / 4)), dim3(NT), 0, st, nc, A, x, y);
    return hipGetLastError();
}

hipError_t launch_gs(int64_t n, double alpha, double sgn, const int32_t* gptr, const GEnt* ents, const double* gv,
                     const double* s, const double* w, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(gs_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, alpha, sgn, gptr, ents, gv, s, w, out);
    return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double* x, const double* y, const double* z, int mode, double* part,
                      double* sc, double* hist, int32_t hist_cap, hipStream_t st)
{
    // the completion counter lives in the scalar block, after the scalars
    unsigned int* done = reinterpret_cast<unsigned int*>(sc + SC_COUNT);
    static_assert(NT == 256, "dot_parts assumes 256 threads per work-group");
    hipLaunchKernelGGL(dot_kernel, dim3(dot_parts(n)), dim3(NT), 0, st, n, x, y, z, mode, part, sc, hist, hist_cap,
                       done);
    return hipGetLastError();
}

hipError_t launch_lumped_local(int32_t nsub, int32_t nbmax, const LumpSub* ls, const int32_t* uptr,
                               const int32_t* uk, const double* sgn, const int32_t* kptr, const int32_t* kcol,
                               const double* kval, const int32_t* mb, const int32_t* dmap, const double* w,
                               double* ylocal, hipStream_t st)
{
    if (nsub <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * 2 * (size_t)std::max(1, nbmax);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)lumped_local_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(lumped_local_kernel, dim3(nsub), dim3(NT), lds, st, ls, uptr, uk, sgn, kptr, kcol, kval, mb,
                       dmap, w, ylocal, nbmax);
    return hipGetLastError();
}

hipError_t launch_block_apply(int64_t n, const int32_t* sb_of, const int32_t* sb_pos, const int32_t* sb_ptr,
                              const int32_t* sb_mem, const int64_t* sb_off, const double* inv, const double* x,
                              double* y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(block_apply_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, sb_of, sb_pos, sb_ptr, sb_mem, sb_off,
                       inv, x, y);
    return hipGetLastError();
}

hipError_t launch_lumped_gather(int64_t n, const int32_t* gptr, const int32_t* gpos, const double* ylocal,
                                double* y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lumped_gather_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, gptr, gpos, ylocal, y);
    return hipGetLastError();
}

hipError_t launch_update_lr(int64_t n, const double* sc, const double* p, const double* q, double* lam, double* r,
                            hipStream_t st)
{
    hipLaunchKernelGGL(update_lr_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, sc, p, q, lam, r);
    return hipGetLastError();
}

hipError_t launch_update_p(int64_t n, int use_beta, const double* sc, const double* y, double* p, hipStream_t st)
{
    hipLaunchKernelGGL(update_p_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, use_beta, sc, y, p);
    return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                        hipStream_t st)
{
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, a, x, b, y, out);
    return hipGetLastError();
}

hipError_t launch_gauss_jordan_inverse(int32_t n, double* A, double* rowk, double* colk, hipStream_t st)
{
    for (int32_t k = 0; k < n; ++k) {
        hipLaunchKernelGGL(gj_copy_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, k, A, rowk, colk);
        hipLaunchKernelGGL(gj_update_kernel, dim3(blocks((int64_t)n * n)), dim3(NT), 0, st, n, k, A, rowk, colk);
    }
    return hipGetLastError();
}

hipError_t launch_permute_out(int64_t n, const int32_t* xperm, const double* x, double* u, hipStream_t st)
{
    hipLaunchKernelGGL(permute_out_kernel, dim3(blocks(n)), dim3(NT), 0, st, n, xperm, x, u);
    return hipGetLastError();
}

hipError_t launch_add_kernel_part(int32_t nsub, const CoarseSub* cs, const double* R, const double* alpha, double* u,
                                  hipStream_t st)
{
    hipLaunchKernelGGL(add_kernel_part, dim3(nsub), dim3(NT), 0, st, cs, R, alpha, u);
    return hipGetLastError();
}

hipError_t launch_load_primal_rhs(int32_t nsub, const int32_t* sub_rowbase, const int32_t* sub_mbase,
                                  const int32_t* xperm, const int32_t* start_rows, const int8_t* signs,
                                  const int32_t* dmap, const double* f, const double* lam, double* x, hipStream_t st)
{
    hipLaunchKernelGGL(load_primal_rhs_kernel, dim3(nsub), dim3(NT), 0, st, sub_rowbase, sub_mbase, xperm,
                       start_rows, signs, dmap, f, lam, x);
    return hipGetLastError();
}

hipError_t launch_first_nonfinite(int prec, const void* x, int64_t n, unsigned long long* first, hipStream_t st)
{
    // the sentinel by a kernel, not a memset node (the call may sit in a graph)
    hipLaunchKernelGGL(set_all_ones_kernel, dim3(1), dim3(1), 0, st, first);
    if (n <= 0) return hipGetLastError();
    const unsigned groups = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 4096);
    if (prec == 0)
        hipLaunchKernelGGL(first_nonfinite_kernel<8>, dim3(groups), dim3(NT), 0, st, x, n, first);
    else if (prec == 1)
        hipLaunchKernelGGL(first_nonfinite_kernel<4>, dim3(groups), dim3(NT), 0, st, x, n, first);
    else
        hipLaunchKernelGGL(first_nonfinite_kernel<2>, dim3(groups), dim3(NT), 0, st, x, n, first);
    return hipGetLastError();
}

}  // namespace fetif
