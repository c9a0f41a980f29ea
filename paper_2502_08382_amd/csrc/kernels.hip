// HIP kernels of the explicit FETI dual operator for gfx950 (CDNA4).
//
//  rhs init     X_i <- P_i B~_i^T on the compact, supernode-blocked X
//  trsm_level   X_i <- L_i^{-1} X_i, one etree height level per launch
//               (right-looking supernodal forward substitution; items of one
//               level touch disjoint RHS column ranges, so no atomics)
//  syrk         F~_i = X_i^T X_i on lower-triangle tiles, summing only the
//               supernodes whose RHS range meets both tiles
//  apply_band   partial symmetric matvec of a row band of the packed triangle
//  gather       q[g] = sum of the band partials of every (subdomain, row)
//               that carries multiplier g, in a fixed order
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace fetif {

namespace {

constexpr int NT = 256;  // threads per work-group (4 wavefronts of 64)

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------- storage conversions

struct bf16_t {
    uint16_t bits;
};

// FP64 -> BF16, round to nearest even.  The FP64 value is first rounded to
// FP32 with round-to-odd (exact when representable, otherwise the truncated
// value with its last bit set), which makes the second rounding to BF16
// equal to a single correct rounding.  Non-finite values keep their class.
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double x)
{
    float f = (float)x;
    if (isfinite(f) && (double)f != x) {
        uint32_t b = __float_as_uint(f);
        if (fabs((double)f) > fabs(x)) b -= 1;  // step toward zero (same sign)
        b |= 1u;
        f = __uint_as_float(b);
    }
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

template <typename T>
__device__ __forceinline__ void store_f(T* p, double v);
template <>
__device__ __forceinline__ void store_f<double>(double* p, double v) { *p = v; }
template <>
__device__ __forceinline__ void store_f<float>(float* p, double v) { *p = (float)v; }
template <>
__device__ __forceinline__ void store_f<bf16_t>(bf16_t* p, double v) { p->bits = f64_to_bf16_rne(v); }

// ---------------------------------------------------------------- fill / rhs

__global__ void fill_zero_kernel(double* __restrict__ x, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) x[i] = 0.0;
}

__global__ void rhs_units_kernel(const RhsUnit* __restrict__ u, int64_t n, double* __restrict__ X)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) X[u[i].off] = u[i].sign;
}

// ---------------------------------------------------------------- TRSM

// One work-group solves one RHS column chunk of one supernode:
//   X_s <- L_ss^{-1} X_s          (column-parallel forward substitution in LDS)
//   X[rows(s)] -= L_rs X_s        (update of the ancestors' rows)
// slot_w (a power of two <= 64) columns are processed; the chunk's own width
// cw <= slot_w, extra columns stay zero.
__global__ __launch_bounds__(NT) void trsm_level_kernel(const TrsmItem* __restrict__ items, int32_t slot_w,
                                                        const DevSN* __restrict__ sns,
                                                        const double* __restrict__ L,
                                                        const int32_t* __restrict__ rows,
                                                        const XRow* __restrict__ xrows,
                                                        double* __restrict__ X)
{
    extern __shared__ double sx[];
    const TrsmItem it = items[blockIdx.x];
    const DevSN s = sns[it.sn];
    const int tid = threadIdx.x;
    const int CW = slot_w;
    const int cw = it.cw;
    const int ns = s.ncols, nr = s.nrows, d = ns + nr;
    const double* __restrict__ P = L + s.lval;
    const int c = tid & (CW - 1);
    const int g = tid / CW;
    const int G = NT / CW;
    for (int idx = tid; idx < ns * CW; idx += NT) {
        int r = idx / CW, cc = idx - r * CW;
        sx[idx] = cc < cw ? X[s.xoff + (int64_t)r * s.w + it.c0 + cc] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < ns; ++k) {
        if (g == 0) sx[k * CW + c] /= P[(int64_t)k * d + k];
        __syncthreads();
        const double xk = sx[k * CW + c];
        const double* __restrict__ colk = P + (int64_t)k * d;
        for (int i = k + 1 + g; i < ns; i += G) sx[i * CW + c] -= colk[i] * xk;
        __syncthreads();
    }
    for (int i = g; i < nr; i += G) {
        double acc = 0.0;
        for (int k = 0; k < ns; ++k) acc += P[(int64_t)k * d + ns + i] * sx[k * CW + c];
        if (c < cw) {
            const int r = rows[s.rowsoff + i];
            const XRow xr = xrows[s.rowbase + r];
            X[xr.off + (s.j0 + it.c0 + c - xr.j0)] -= acc;
        }
    }
    for (int idx = tid; idx < ns * CW; idx += NT) {
        int r = idx / CW, cc = idx - r * CW;
        if (cc < cw) X[s.xoff + (int64_t)r * s.w + it.c0 + cc] = sx[idx];
    }
}

// ---------------------------------------------------------------- SYRK

constexpr int ST = 64;   // output tile edge
constexpr int SK = 16;   // rows of X per LDS stage

template <typename T>
__global__ __launch_bounds__(NT) void syrk_kernel(const SyrkTile* __restrict__ tiles,
                                                  const int32_t* __restrict__ lists,
                                                  const DevSN* __restrict__ sns,
                                                  const double* __restrict__ X, T* __restrict__ F)
{
    __shared__ double sa[SK][ST + 1];
    __shared__ double sb[SK][ST + 1];
    const SyrkTile t = tiles[blockIdx.x];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int ca0 = t.ta * ST, cb0 = t.tb * ST;
    for (int li = t.list0; li < t.list1; ++li) {
        const DevSN s = sns[lists[li]];
        for (int k0 = 0; k0 < s.ncols; k0 += SK) {
            for (int idx = tid; idx < SK * ST; idx += NT) {
                const int kk = idx / ST, cc = idx - kk * ST;
                const int k = k0 + kk;
                const int ja = ca0 + cc - s.j0, jb = cb0 + cc - s.j0;
                const bool kin = k < s.ncols;
                const double* xr = X + s.xoff + (int64_t)k * s.w;
                sa[kk][cc] = (kin && ja >= 0 && ja < s.w) ? xr[ja] : 0.0;
                sb[kk][cc] = (kin && jb >= 0 && jb < s.w) ? xr[jb] : 0.0;
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < SK; ++kk) {
                double ra[4], rb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) ra[i] = sa[kk][ty * 4 + i];
#pragma unroll
                for (int j = 0; j < 4; ++j) rb[j] = sb[kk][tx * 4 + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] += ra[i] * rb[j];
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = ca0 + ty * 4 + i;
        if (row >= t.m) continue;
        T* frow = F + t.fbase + packed_row_offset(row, (int64_t)(16 / sizeof(T)));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = cb0 + tx * 4 + j;
            if (col <= row) store_f<T>(frow + col, acc[i][j]);
        }
    }
}

// ---------------------------------------------------------------- apply

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    using type = double;
};
template <>
struct Acc<float> {
    using type = float;
};
template <>
struct Acc<bf16_t> {
    using type = float;
};

template <typename T, int VEC>
__device__ __forceinline__ void unpack(const uint4& raw, typename Acc<T>::type (&v)[VEC]);
template <>
__device__ __forceinline__ void unpack<double, 2>(const uint4& raw, double (&v)[2])
{
    v[0] = __hiloint2double((int)raw.y, (int)raw.x);
    v[1] = __hiloint2double((int)raw.w, (int)raw.z);
}
template <>
__device__ __forceinline__ void unpack<float, 4>(const uint4& raw, float (&v)[4])
{
    v[0] = __uint_as_float(raw.x);
    v[1] = __uint_as_float(raw.y);
    v[2] = __uint_as_float(raw.z);
    v[3] = __uint_as_float(raw.w);
}
template <>
__device__ __forceinline__ void unpack<bf16_t, 8>(const uint4& raw, float (&v)[8])
{
    const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = __uint_as_float(w[k] << 16);
        v[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NTL>
__device__ __forceinline__ uint4 load16(const void* p)
{
    if constexpr (NTL) {
        u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const uint4*>(p);
    }
}

// One work-group handles one band of rows [r0, r1) of a packed lower
// triangle: every stored element F[r][c] (c <= r) contributes F[r][c] p[c] to
// row r (a dot product, reduced across the wavefront) and, for c < r,
// F[r][c] p[r] to row c (kept in per-lane registers).  The band writes its
// partial vector z[0..r1).  Lanes read 16-byte vectors of consecutive
// columns, so a wavefront streams 1 KiB of a row per load; a wavefront
// takes ROWS consecutive rows per pass (their loads are in flight together).
template <typename T, int NCH, int ROWS, bool NTL>
__global__ __launch_bounds__(NT) void apply_band_kernel(const Band* __restrict__ bands,
                                                        const T* __restrict__ F,
                                                        const double* __restrict__ lam,
                                                        const int32_t* __restrict__ dmap,
                                                        typename Acc<T>::type* __restrict__ z)
{
    using A = typename Acc<T>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int CH = 64 * VEC;  // columns per chunk
    constexpr int CAP = NCH * CH;
    __shared__ A sp[CAP];   // p = lambda[D_i] (sorted order); later the partial sums
    __shared__ A srow[CAP]; // row dot products of the band
    const Band b = bands[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int cidx = tid; cidx < b.r1; cidx += NT) sp[cidx] = (A)lam[dmap[b.dbase + cidx]];
    __syncthreads();
    A y[NCH][VEC];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int e = 0; e < VEC; ++e) y[ch][e] = (A)0;
    for (int r = b.r0 + ROWS * wv; r < b.r1; r += 4 * ROWS) {
        const T* __restrict__ rowp = F + b.fbase + packed_row_offset(r, VEC);
        uint4 raw[ROWS][NCH];
        int rr[ROWS];
        const T* rp[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            rr[k] = (r + k < b.r1) ? r + k : -1;   // -1: no such row, loads masked off
            rp[k] = k == 0 ? rowp : rp[k - 1] + VEC * ((r + k - 1) / VEC + 1);
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int col = ch * CH + lane * VEC;
                raw[k][ch] = col <= rr[k] ? load16<NTL>(rp[k] + col) : make_uint4(0, 0, 0, 0);
            }
        A pr[ROWS], dot[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            pr[k] = rr[k] >= 0 ? sp[rr[k]] : (A)0;
            dot[k] = (A)0;
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int col = ch * CH + lane * VEC;
            if (col <= rr[ROWS - 1] || col <= rr[0]) {
                A pc[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) pc[e] = sp[col + e];
#pragma unroll
                for (int k = 0; k < ROWS; ++k) {
                    if (col <= rr[k]) {
                        A v[VEC];
                        unpack<T, VEC>(raw[k][ch], v);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const int cc = col + e;
                            if (cc <= rr[k]) {
                                dot[k] += v[e] * pc[e];
                                if (cc < rr[k]) y[ch][e] += v[e] * pr[k];
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k) dot[k] = wave_sum(dot[k]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < ROWS; ++k)
                if (rr[k] >= 0) srow[rr[k] - b.r0] = dot[k];
        }
    }
    __syncthreads();
    // sp is free now: sum the four wavefronts' column partials in order
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int cc = ch * CH + lane * VEC + e;
                    if (cc < b.r1) sp[cc] = (w == 0 ? (A)0 : sp[cc]) + y[ch][e];
                }
        }
        __syncthreads();
    }
    for (int cidx = tid; cidx < b.r1; cidx += NT)
        z[b.zoff + cidx] = sp[cidx] + (cidx >= b.r0 ? srow[cidx - b.r0] : (A)0);
}

template <typename A>
__global__ __launch_bounds__(NT) void gather_kernel(int64_t n_lambda, const int32_t* __restrict__ gptr,
                                                    const GatherEnt* __restrict__ ents,
                                                    const int64_t* __restrict__ band_zoff,
                                                    const A* __restrict__ z, double* __restrict__ q)
{
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n_lambda) return;
    double acc = 0.0;
    for (int32_t e = gptr[g]; e < gptr[g + 1]; ++e) {
        const GatherEnt E = ents[e];
        for (int32_t bb = E.b0; bb < E.b1; ++bb) acc += (double)z[band_zoff[bb] + E.a];
    }
    q[g] = acc;
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_fill_zero(double* x, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + NT - 1) / NT;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(NT), 0, st, x, n);
    return hipGetLastError();
}

hipError_t launch_rhs_units(const RhsUnit* u, int64_t n, double* X, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rhs_units_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, u, n, X);
    return hipGetLastError();
}

hipError_t launch_trsm_level(const TrsmItem* items, int32_t nitems, int32_t slot_w, int32_t max_ns,
                             const DevSN* sns, const double* L, const int32_t* rows, const XRow* xrows,
                             double* X, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    size_t lds = sizeof(double) * (size_t)max_ns * slot_w;
    hipLaunchKernelGGL(trsm_level_kernel, dim3(nitems), dim3(NT), lds, st, items, slot_w, sns, L, rows,
                       xrows, X);
    return hipGetLastError();
}

hipError_t launch_syrk(int prec, const SyrkTile* tiles, int32_t ntiles, const int32_t* lists,
                       const DevSN* sns, const double* X, void* F, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(syrk_kernel<double>, dim3(ntiles), dim3(NT), 0, st, tiles, lists, sns, X,
                           (double*)F);
    else if (prec == 1)
        hipLaunchKernelGGL(syrk_kernel<float>, dim3(ntiles), dim3(NT), 0, st, tiles, lists, sns, X,
                           (float*)F);
    else
        hipLaunchKernelGGL(syrk_kernel<bf16_t>, dim3(ntiles), dim3(NT), 0, st, tiles, lists, sns, X,
                           (bf16_t*)F);
    return hipGetLastError();
}

template <typename T, int NCH, int ROWS, bool NTL>
static void apply_launch(const Band* bands, int32_t nbands, const T* f, const double* lam, const int32_t* dmap,
                         typename Acc<T>::type* z, hipStream_t st)
{
    // a band keeps NCH * 64 * VEC columns of p and of the row sums in LDS;
    // only instantiate shapes whose capacity stays within 4096 columns
    if constexpr (NCH * 64 * (16 / (int)sizeof(T)) <= 4096)
        hipLaunchKernelGGL((apply_band_kernel<T, NCH, ROWS, NTL>), dim3(nbands), dim3(NT), 0, st, bands, f, lam,
                           dmap, z);
}

template <typename T, int ROWS, bool NTL>
static hipError_t apply_dispatch_nch(int nch, const Band* bands, int32_t nbands, const void* F, const double* lam,
                                     const int32_t* dmap, void* z, hipStream_t st)
{
    using A = typename Acc<T>::type;
    const T* f = (const T*)F;
    A* zz = (A*)z;
    if (nch * 64 * (16 / (int)sizeof(T)) > 4096) return hipErrorInvalidValue;
    switch (nch) {
    case 1: apply_launch<T, 1, ROWS, NTL>(bands, nbands, f, lam, dmap, zz, st); break;
    case 2: apply_launch<T, 2, ROWS, NTL>(bands, nbands, f, lam, dmap, zz, st); break;
    case 4: apply_launch<T, 4, ROWS, NTL>(bands, nbands, f, lam, dmap, zz, st); break;
    case 8: apply_launch<T, 8, ROWS, NTL>(bands, nbands, f, lam, dmap, zz, st); break;
    case 16: apply_launch<T, 16, ROWS, NTL>(bands, nbands, f, lam, dmap, zz, st); break;
    case 32: apply_launch<T, 32, ROWS, NTL>(bands, nbands, f, lam, dmap, zz, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t apply_dispatch(int nch, int rows, bool ntl, const Band* bands, int32_t nbands, const void* F,
                                 const double* lam, const int32_t* dmap, void* z, hipStream_t st)
{
    if (rows == 1)
        return ntl ? apply_dispatch_nch<T, 1, true>(nch, bands, nbands, F, lam, dmap, z, st)
                   : apply_dispatch_nch<T, 1, false>(nch, bands, nbands, F, lam, dmap, z, st);
    if (rows == 2)
        return ntl ? apply_dispatch_nch<T, 2, true>(nch, bands, nbands, F, lam, dmap, z, st)
                   : apply_dispatch_nch<T, 2, false>(nch, bands, nbands, F, lam, dmap, z, st);
    return hipErrorInvalidValue;
}

hipError_t launch_apply_band(int prec, int nch, int rows, bool ntl, const Band* bands, int32_t nbands,
                             const void* F, const double* lam, const int32_t* dmap, void* z, hipStream_t st)
{
    if (nbands <= 0) return hipSuccess;
    if (prec == 0) return apply_dispatch<double>(nch, rows, ntl, bands, nbands, F, lam, dmap, z, st);
    if (prec == 1) return apply_dispatch<float>(nch, rows, ntl, bands, nbands, F, lam, dmap, z, st);
    return apply_dispatch<bf16_t>(nch, rows, ntl, bands, nbands, F, lam, dmap, z, st);
}

hipError_t launch_gather(int prec, int64_t n_lambda, const int32_t* gptr, const GatherEnt* ents,
                         const int64_t* band_zoff, const void* z, double* q, hipStream_t st)
{
    if (n_lambda <= 0) return hipSuccess;
    dim3 grid((unsigned)((n_lambda + NT - 1) / NT));
    if (prec == 0)
        hipLaunchKernelGGL(gather_kernel<double>, grid, dim3(NT), 0, st, n_lambda, gptr, ents, band_zoff,
                           (const double*)z, q);
    else
        hipLaunchKernelGGL(gather_kernel<float>, grid, dim3(NT), 0, st, n_lambda, gptr, ents, band_zoff,
                           (const float*)z, q);
    return hipGetLastError();
}

}  // namespace fetif
