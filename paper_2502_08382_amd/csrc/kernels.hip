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
#include <mutex>

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

// v from the lane selected by a DPP pattern within each row of 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp_get(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_get(double v)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sums of R per-lane partials d[0..R) over the 64 lanes of a wavefront
// (R = 1, 2 or 4).  The first log2(R) butterfly steps (lane distance 32,
// then 16) each hand half of the still-separate sums to the partner lane,
// so lane l ends with the sum of d[(l >> (6 - log2 R))], i.e. sum k sits in
// lanes [k * 64 / R, (k + 1) * 64 / R).  The steps inside a row of 16 lanes
// use DPP (quad swaps, then half-row and row mirrors) instead of LDS
// permutes.  Fixed order: the result is bitwise reproducible.
template <int R, typename A>
__device__ __forceinline__ A rows_wave_sum(const A (&d)[R], int lane)
{
    static_assert(R == 1 || R == 2 || R == 4, "R in {1,2,4}");
    A v;
    if constexpr (R == 1) {
        v = d[0];
        v += __shfl_xor(v, 32, 64);
        v += __shfl_xor(v, 16, 64);
    } else if constexpr (R == 2) {
        const bool hi = (lane & 32) != 0;
        v = (hi ? d[1] : d[0]) + __shfl_xor(hi ? d[0] : d[1], 32, 64);
        v += __shfl_xor(v, 16, 64);
    } else {
        const bool hi = (lane & 32) != 0;
        A k0 = (hi ? d[2] : d[0]) + __shfl_xor(hi ? d[0] : d[2], 32, 64);
        A k1 = (hi ? d[3] : d[1]) + __shfl_xor(hi ? d[1] : d[3], 32, 64);
        const bool h16 = (lane & 16) != 0;
        v = (h16 ? k1 : k0) + __shfl_xor(h16 ? k0 : k1, 16, 64);
    }
    v += dpp_get<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_get<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_get<0x141>(v);  // row_half_mirror: quads 0<->1, 2<->3
    v += dpp_get<0x140>(v);  // row_mirror: half-rows swapped
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

constexpr int kTrsmMaxNb = 6;   // 16-column blocks of the widest TRSM panel (96 columns)

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operand layout on gfx950 (lane l, q = l / 16,
// j = l % 16): A holds A[j][q], B holds B[q][j], and accumulator register r
// holds D[q + 4r][j].  Register r of a product is therefore exactly the B
// operand of k-step r of the next product, with no data movement.
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// 8 bytes per lane from a buffer descriptor covering [base, base + nbytes):
// lanes whose bytes fall outside (a negative offset wraps to a large one)
// read zero, so the loads need no branches.
__device__ __forceinline__ double load8_range(const double* base, uint32_t nbytes, int lane_off)
{
    __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)nbytes, 0x00020000);
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, 0, 0);
    return __hiloint2double((int)v.y, (int)v.x);
}

// Inverse of one 16x16 lower-triangular diagonal block of a supernode panel
// (rows/columns beyond the supernode are the identity).  Thread j of the
// block forms column j by forward substitution.  Stored column-major.
__global__ __launch_bounds__(NT) void diag_inverse_kernel(const InvItem* __restrict__ items, int32_t nitems,
                                                          const DevSN* __restrict__ sns,
                                                          const double* __restrict__ L,
                                                          double* __restrict__ Linv)
{
    const int t = blockIdx.x * NT + threadIdx.x;
    const int item = t >> 4, j = t & 15;
    if (item >= nitems) return;
    const InvItem it = items[item];
    const DevSN s = sns[it.sn];
    const int ns = s.ncols, d = s.ncols + s.nrows, base = it.rb * 16;
    const double* __restrict__ P = L + s.lval;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int gi = base + i;
        double v = (i == j) ? 1.0 : 0.0;
        if (gi < ns) {
#pragma unroll
            for (int k = 0; k < i; ++k) v -= P[(int64_t)(base + k) * d + gi] * x[k];
            v /= P[(int64_t)gi * d + gi];
        }
        x[i] = v;
    }
    double* out = Linv + s.linv + (int64_t)it.rb * 256 + j * 16;
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = x[i];
}

// One work-group solves one RHS column chunk (up to 16 W columns) of one
// supernode panel s, in two phases:
//  1. each of its W wavefronts owns 16 columns and, alone,
//       for each 16-row block rb:  acc = X[rb] - sum_{kb<rb} L[rb,kb] X[kb]
//                                  X[rb] = inv(L[rb,rb]) acc          (MFMA)
//     keeping the solved blocks in LDS in B-operand order;
//  2. after a barrier the below rows are split by 16-row blocks over the
//     wavefronts; each computes X[rows] -= L[rows, s] X_s for all of the
//     chunk's columns, so every loaded L operand feeds one MFMA per 16-column
//     block (independent accumulator chains) and is read once per work-group.
// rowoff[i] is the X offset of below row i minus the first RHS column of its
// range.  Items of one level touch disjoint RHS column ranges, so the
// updates need no atomics.
template <int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(W == 4 ? 2 : 3))) void trsm_level_kernel(const TrsmItem* __restrict__ items, int32_t nbmax,
                                  const DevSN* __restrict__ sns, const double* __restrict__ L,
                                  const double* __restrict__ Linv, const int64_t* __restrict__ rowoff,
                                  double* __restrict__ X)
{
    extern __shared__ double smem[];
    const TrsmItem it = items[blockIdx.x];
    if (it.cw == 0) return;  // padding item of the die-aware order (whole work-group)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int q = lane >> 4, j = lane & 15;
    const DevSN s = sns[it.sn];
    const int ns = s.ncols, nr = s.nrows, d = s.ld;
    const int nb = (ns + 15) >> 4;
    const double* __restrict__ P = L + s.lval;
    double* __restrict__ sx0 = smem;                     // [W][nbmax * 4][64]
    double* __restrict__ sx = smem + (size_t)wv * nbmax * 256;
    const int cbeg = wv * 16;
    if (cbeg < it.cw) {
        const int col = it.c0 + cbeg + j;                // column relative to j0
        const bool cv = (cbeg + j) < it.cw;
        const double* __restrict__ PI = Linv + s.linv;
        // Row block rb's operands -- the chain's L entries, the diagonal
        // inverse and the X rows -- are requested one row block ahead,
        // during block rb - 1's chain.  The loads go through buffer
        // descriptors over the panel, its inverses and its X block, so an
        // entry outside them (a lane past the panel, the block after the
        // last) reads zero without a branch and the compiler waits only for
        // the block in use.
        double* __restrict__ xsb = X + s.xoff;           // X_s[row][col] at row * w + col
        const uint32_t l_bytes = (uint32_t)ns * (uint32_t)d * 8u;
        const uint32_t pi_bytes = (uint32_t)nb * 256u * 8u;
        const uint32_t x_bytes = (uint32_t)ns * (uint32_t)s.w * 8u;
        constexpr int kOut = 0x7ffffff0;                 // beyond every range
        auto load_ops = [&](int rb, double (&ap)[kTrsmMaxNb - 1][4], double (&pi)[4], d4& xv) {
            const int arow = rb * 16 + j;
            const bool av = arow < ns;
#pragma unroll
            for (int kb = 0; kb < kTrsmMaxNb - 1; ++kb)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int kc = kb * 16 + 4 * kk + q;
                    const int off = (kb < rb && av) ? (kc * d + arow) * 8 : kOut;
                    ap[kb][kk] = -load8_range(P, l_bytes, off);
                }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) pi[kk] = load8_range(PI, pi_bytes, (rb * 256 + (4 * kk + q) * 16 + j) * 8);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rb * 16 + q + 4 * r;
                xv[r] = load8_range(xsb, x_bytes, (cv && row < ns) ? (row * s.w + col) * 8 : kOut);
            }
        };
        double ap[kTrsmMaxNb - 1][4], pi[4];
        d4 xin;
        load_ops(0, ap, pi, xin);
        for (int rb = 0; rb < nb; ++rb) {
            d4 acc = xin;
            double apn[kTrsmMaxNb - 1][4], pin[4];
            load_ops(rb + 1, apn, pin, xin);
#pragma unroll
            for (int kb = 0; kb < kTrsmMaxNb - 1; ++kb) {
                if (kb >= rb) break;                     // wavefront-uniform
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) acc = mfma16(ap[kb][kk], sx[(kb * 4 + kk) * 64 + lane], acc);
            }
            d4 xn = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) xn = mfma16(pi[kk], acc[kk], xn);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sx[(rb * 4 + r) * 64 + lane] = xn[r];
                const int row = rb * 16 + q + 4 * r;
                if (cv && row < ns) xsb[(int64_t)row * s.w + col] = xn[r];
            }
#pragma unroll
            for (int kb = 0; kb < kTrsmMaxNb - 1; ++kb)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) ap[kb][kk] = apn[kb][kk];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) pi[kk] = pin[kk];
        }
    } else {
        // no columns: a zero block, so phase 2 may multiply every block
        for (int idx = lane; idx < nb * 256; idx += 64) sx[idx] = 0.0;
    }
    __syncthreads();
    const int64_t jbase = (int64_t)s.j0 + it.c0;
    // row offsets of the wavefront's next row block are requested one block
    // ahead, so a block's X addresses do not wait for them
    int64_t ro[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = wv * 16 + q + 4 * r;
        ro[r] = i < nr ? rowoff[s.rowsoff + i] : 0;
    }
    for (int rb = wv; rb * 16 < nr; rb += W) {
        // the target X values first: their loads are in flight while the
        // MFMA chain below runs
        double* xr[4];
        double xv[4][W];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = rb * 16 + q + 4 * r;
            xr[r] = i < nr ? X + ro[r] + jbase : nullptr;
#pragma unroll
            for (int c = 0; c < W; ++c) xv[r][c] = (xr[r] && c * 16 + j < it.cw) ? xr[r][c * 16 + j] : 0.0;
        }
        d4 acc[W];
#pragma unroll
        for (int c = 0; c < W; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = (rb + W) * 16 + q + 4 * r;
            ro[r] = i < nr ? rowoff[s.rowsoff + i] : 0;
        }
        const int arow = ns + rb * 16 + j;
        const bool av = arow < ns + nr;
        // the row block's L operands of a panel of up to kTrsmMaxNb blocks,
        // requested together (one memory latency per row block)
        double a[kTrsmMaxNb][4];
#pragma unroll
        for (int kb = 0; kb < kTrsmMaxNb; ++kb)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int kc = kb * 16 + 4 * kk + q;
                a[kb][kk] = (kb < nb && av && kc < ns) ? P[(int64_t)kc * d + arow] : 0.0;
            }
#pragma unroll
        for (int kb = 0; kb < kTrsmMaxNb; ++kb) {
            if (kb >= nb) break;                         // wavefront-uniform
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int c = 0; c < W; ++c)
                    acc[c] = mfma16(a[kb][kk], sx0[((size_t)c * nbmax * 4 + kb * 4 + kk) * 64 + lane], acc[c]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (xr[r]) {
#pragma unroll
                for (int c = 0; c < W; ++c)
                    if (c * 16 + j < it.cw) xr[r][c * 16 + j] = xv[r][c] - acc[c][r];
            }
    }
}

// ---------------------------------------------------------------- TRSM path

// Backward supernodal solve of the TRSM path (Sec. IV-C, two TRSMs and an
// SpMM): Z_i = L_i^{-T} X_i with X_i the forward solution, Z_i dense
// (n_i x m_i, row-major, columns in the sorted multiplier order).  One
// work-group takes 16 W of the m_i columns of one column panel p (record
// `pans[it.sn]`: ncols panel columns, nrows rows below them -- the later
// columns of its supernode, then the supernode's below rows --, ld, the
// panel's L and inverse offsets, its compact X block (xoff, j0, w: X is
// zero outside the RHS range [j0, j0 + w)), zrow[rowsoff + k] the Z offset
// of row k of the panel (the ncols panel rows, then the below rows), and
// pad = m_i); wavefront wv owns 16 of them.  Levels run from the root
// down, so every row below the panel is solved already:
//   acc = X[panel rows] - L[below, panel]^T Z[below]   (MFMA over the below rows, 16 at a time)
//   rb = nb-1 .. 0:  Z[rb] = inv(L[rb,rb])^T (acc[rb] - sum_{kb > rb} L[kb,rb]^T Z[kb])
// With the accumulator layout (register r holds rows q + 4r), register r
// of a solved block is the B operand of k-step r of the next product.
template <int W>
__global__ __launch_bounds__(64 * W) void trsm_bwd_level_kernel(const TrsmItem* __restrict__ items,
                                                                const DevSN* __restrict__ pans,
                                                                const double* __restrict__ L,
                                                                const double* __restrict__ Linv,
                                                                const int64_t* __restrict__ zrow,
                                                                const double* __restrict__ X,
                                                                double* __restrict__ Z)
{
    const TrsmItem it = items[blockIdx.x];
    if (it.cw == 0) return;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int q = lane >> 4, j = lane & 15;
    if (wv * 16 >= it.cw) return;
    const DevSN s = pans[it.sn];
    const int ns = s.ncols, nr = s.nrows, d = s.ld;
    const int nb = (ns + 15) >> 4;
    const double* __restrict__ P = L + s.lval;
    const int64_t* __restrict__ zr = zrow + s.rowsoff;
    const int col = it.c0 + wv * 16 + j;               // column of Z (sorted multiplier order)
    const bool cv = wv * 16 + j < it.cw;
    const bool xin = cv && col >= s.j0 && col < s.j0 + s.w;
    d4 acc[kTrsmMaxNb];
#pragma unroll
    for (int kb = 0; kb < kTrsmMaxNb; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = kb * 16 + q + 4 * r;
            acc[kb][r] = (kb < nb && xin && row < ns) ? X[s.xoff + (int64_t)row * s.w + (col - s.j0)] : 0.0;
        }
    // below rows, 16 per step (4 k-steps of 4): the next step's Z rows and
    // L operands are requested before the current step's MFMAs
    auto load_step = [&](int k0, double (&zb)[4], double (&a)[kTrsmMaxNb][4]) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = k0 + 4 * kk + q;
            zb[kk] = (k < nr && cv) ? Z[zr[ns + k] + col] : 0.0;
#pragma unroll
            for (int kb = 0; kb < kTrsmMaxNb; ++kb)
                a[kb][kk] = (kb < nb && k < nr && kb * 16 + j < ns) ? -P[(int64_t)(kb * 16 + j) * d + ns + k] : 0.0;
        }
    };
    if (nr > 0) {
        double zb[4], a[kTrsmMaxNb][4];
        load_step(0, zb, a);
        for (int k0 = 0; k0 < nr; k0 += 16) {
            double zbn[4], an[kTrsmMaxNb][4];
            load_step(k0 + 16, zbn, an);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int kb = 0; kb < kTrsmMaxNb; ++kb) {
                    if (kb >= nb) break;                 // wavefront-uniform
                    acc[kb] = mfma16(a[kb][kk], zb[kk], acc[kb]);
                }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                zb[kk] = zbn[kk];
#pragma unroll
                for (int kb = 0; kb < kTrsmMaxNb; ++kb) a[kb][kk] = an[kb][kk];
            }
        }
    }
    // the panel's own rows, last row block first
    const double* __restrict__ PI = Linv + s.linv;
    d4 zs[kTrsmMaxNb];
#pragma unroll
    for (int rb = kTrsmMaxNb - 1; rb >= 0; --rb) {
        if (rb >= nb) continue;                          // wavefront-uniform
        d4 t = acc[rb];
#pragma unroll
        for (int kb = rb + 1; kb < kTrsmMaxNb; ++kb) {
            if (kb >= nb) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = kb * 16 + q + 4 * r, cl = rb * 16 + j;
                const double av = (row < ns && cl < ns) ? -P[(int64_t)cl * d + row] : 0.0;
                t = mfma16(av, zs[kb][r], t);
            }
        }
        d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 4; ++r) z = mfma16(PI[rb * 256 + j * 16 + q + 4 * r], t[r], z);
        zs[rb] = z;
    }
    if (cv) {
#pragma unroll
        for (int rb = 0; rb < kTrsmMaxNb; ++rb) {
            if (rb >= nb) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rb * 16 + q + 4 * r;
                if (row < ns) Z[zr[row] + col] = zs[rb][r];
            }
        }
    }
}

// F~_i = B~_i P_i^T Z_i, the SpMM of the TRSM path: row a (sorted order) of
// F~_i is sign_a times row start_a of Z_i; its columns 0..a go to the packed
// triangle in the storage precision.  One wavefront per row of every F~_i
// (global sorted row g of subdomain i: sub_m[i] <= g < sub_m[i + 1]).
template <typename T>
__global__ __launch_bounds__(NT) void tri_from_z_kernel(int32_t nsub, int64_t nrows, const int32_t* __restrict__ sub_m,
                                                        const int32_t* __restrict__ start_rows,
                                                        const int8_t* __restrict__ signs,
                                                        const int64_t* __restrict__ zbase,
                                                        const int64_t* __restrict__ fbase,
                                                        const double* __restrict__ Z, T* __restrict__ F)
{
    const int64_t g = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= nrows) return;
    int lo = 0, hi = nsub;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sub_m[mid] <= g) lo = mid;
        else hi = mid;
    }
    const int a = (int)(g - sub_m[lo]);
    const int m = sub_m[lo + 1] - sub_m[lo];
    constexpr int RA = kRowAlignBytes / sizeof(T);
    const double sg = (double)signs[g];
    const double* __restrict__ zrw = Z + zbase[lo] + (int64_t)start_rows[g] * m;
    T* __restrict__ fr = F + fbase[lo] + packed_row_offset(a, RA);
    for (int b = lane; b <= a; b += 64) store_f<T>(fr + b, sg * zrw[b]);
}

// ---------------------------------------------------------------- TRSV

// x <- P B~^T D v for every subdomain (one work-group per subdomain).  The
// subdomain's local multipliers are sorted by their permuted DOF, so equal
// DOFs are adjacent: the first column of each run sums the run (fixed order).
template <int NRHS>
__global__ __launch_bounds__(NT) void scatter_dual_kernel(const int32_t* __restrict__ sub_rowbase,
                                                          const int32_t* __restrict__ sub_mbase,
                                                          const int32_t* __restrict__ start_rows,
                                                          const int8_t* __restrict__ signs,
                                                          const int32_t* __restrict__ dmap,
                                                          const double* __restrict__ v0,
                                                          const double* __restrict__ v1, double* __restrict__ x)
{
    const int i = blockIdx.x;
    const int rb = sub_rowbase[i], r1 = sub_rowbase[i + 1];
    const int m0 = sub_mbase[i], m1 = sub_mbase[i + 1];
    for (int r = rb + threadIdx.x; r < r1; r += NT)
#pragma unroll
        for (int k = 0; k < NRHS; ++k) x[(int64_t)r * NRHS + k] = 0.0;
    __syncthreads();
    for (int a = m0 + threadIdx.x; a < m1; a += NT) {
        const int row = start_rows[a];
        if (a > m0 && start_rows[a - 1] == row) continue;
        double acc0 = 0.0, acc1 = 0.0;
        for (int b = a; b < m1 && start_rows[b] == row; ++b) {
            const double sg = (double)signs[b];
            acc0 += sg * v0[dmap[b]];
            if (NRHS == 2) acc1 += sg * v1[dmap[b]];
        }
        x[(int64_t)(rb + row) * NRHS] = acc0;
        if (NRHS == 2) x[(int64_t)(rb + row) * NRHS + 1] = acc1;
    }
}

// Forward substitution of one supernode per work-group (multifrontal):
//   front = [x_s ; 0] + extend-add of the children's update vectors
//   x_s  = L_ss^{-1} front_s        (16-row blocks through inv(L_kk))
//   u_s  = front_r - L_rs x_s       (update vector for the parent)
// Children are added one after another, so sums have a fixed order.
template <int NRHS>
__global__ __launch_bounds__(NT) void trsv_forward_kernel(const int32_t* __restrict__ sn_list,
                                                          const DevSN* __restrict__ sns,
                                                          const double* __restrict__ L,
                                                          const double* __restrict__ Linv,
                                                          const int32_t* __restrict__ child_ptr,
                                                          const int32_t* __restrict__ child_idx,
                                                          const int32_t* __restrict__ relpos,
                                                          double* __restrict__ u, double* __restrict__ x)
{
    extern __shared__ double fr[];
    __shared__ double xb[16 * NRHS];
    const int sid = sn_list[blockIdx.x];
    const DevSN s = sns[sid];
    const int tid = threadIdx.x;
    const int ns = s.ncols, nr = s.nrows, d = ns + nr;
    const double* __restrict__ P = L + s.lval;
    double* __restrict__ xs = x + (int64_t)(s.rowbase + s.first) * NRHS;
    for (int idx = tid; idx < d * NRHS; idx += NT) fr[idx] = idx < ns * NRHS ? xs[idx] : 0.0;
    __syncthreads();
    for (int ci = child_ptr[sid]; ci < child_ptr[sid + 1]; ++ci) {
        const DevSN c = sns[child_idx[ci]];
        for (int idx = tid; idx < c.nrows * NRHS; idx += NT) {
            const int i = idx / NRHS, k = idx - i * NRHS;
            fr[relpos[c.rowsoff + i] * NRHS + k] += u[c.rowsoff * NRHS + idx];
        }
        __syncthreads();
    }
    const int nb = (ns + 15) >> 4;
    for (int rb = 0; rb < nb; ++rb) {
        const int b0 = rb * 16, bn = min(16, ns - b0);
        if (tid < 16 * NRHS) {
            const int i = tid / NRHS, k = tid - i * NRHS;
            double acc = 0.0;
            if (i < bn) {
                const double* li = Linv + s.linv + (int64_t)rb * 256 + i;  // Linv[i][kk] at kk*16 + i
                for (int kk = 0; kk < bn; ++kk) acc += li[kk * 16] * fr[(b0 + kk) * NRHS + k];
            }
            xb[tid] = acc;
        }
        __syncthreads();
        if (tid < 16 * NRHS && tid / NRHS < bn) fr[b0 * NRHS + tid] = xb[tid];
        // update every later row (diagonal part and off-diagonal rows)
        for (int i = b0 + bn + tid; i < d; i += NT) {
            double a0 = 0.0, a1 = 0.0;
            for (int kk = 0; kk < bn; ++kk) {
                const double l = P[(int64_t)(b0 + kk) * d + i];
                a0 += l * xb[kk * NRHS];
                if (NRHS == 2) a1 += l * xb[kk * NRHS + 1];
            }
            fr[i * NRHS] -= a0;
            if (NRHS == 2) fr[i * NRHS + 1] -= a1;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < ns * NRHS; idx += NT) xs[idx] = fr[idx];
    for (int idx = tid; idx < nr * NRHS; idx += NT) u[s.rowsoff * NRHS + idx] = fr[ns * NRHS + idx];
}

// Backward substitution of one supernode per work-group (ancestors first):
//   x_s = L_ss^{-T} (y_s - L_rs^T x[rows(s)])
template <int NRHS>
__global__ __launch_bounds__(NT) void trsv_backward_kernel(const int32_t* __restrict__ sn_list,
                                                           const DevSN* __restrict__ sns,
                                                           const double* __restrict__ L,
                                                           const double* __restrict__ Linv,
                                                           const int32_t* __restrict__ rows,
                                                           double* __restrict__ x)
{
    extern __shared__ double fr[];  // ns*NRHS solution part, then nr*NRHS ancestor values
    __shared__ double xb[16 * NRHS];
    const int sid = sn_list[blockIdx.x];
    const DevSN s = sns[sid];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ns = s.ncols, nr = s.nrows, d = ns + nr;
    const double* __restrict__ P = L + s.lval;
    double* __restrict__ xs = x + (int64_t)(s.rowbase + s.first) * NRHS;
    double* __restrict__ xr = fr + ns * NRHS;
    for (int idx = tid; idx < ns * NRHS; idx += NT) fr[idx] = xs[idx];
    for (int idx = tid; idx < nr * NRHS; idx += NT) {
        const int i = idx / NRHS, k = idx - i * NRHS;
        xr[idx] = x[(int64_t)(s.rowbase + rows[s.rowsoff + i]) * NRHS + k];
    }
    __syncthreads();
    // y_s -= L_rs^T x_r: column k of the panel against the ancestor values
    for (int k = wv; k < ns; k += NT / 64) {
        double a0 = 0.0, a1 = 0.0;
        for (int i = lane; i < nr; i += 64) {
            const double l = P[(int64_t)k * d + ns + i];
            a0 += l * xr[i * NRHS];
            if (NRHS == 2) a1 += l * xr[i * NRHS + 1];
        }
        a0 = wave_sum(a0);
        if (NRHS == 2) a1 = wave_sum(a1);
        if (lane == 0) {
            fr[k * NRHS] -= a0;
            if (NRHS == 2) fr[k * NRHS + 1] -= a1;
        }
    }
    __syncthreads();
    const int nb = (ns + 15) >> 4;
    for (int rb = nb - 1; rb >= 0; --rb) {
        const int b0 = rb * 16, bn = min(16, ns - b0);
        if (tid < 16 * NRHS) {
            const int i = tid / NRHS, k = tid - i * NRHS;
            double acc = 0.0;
            if (i < bn) {
                const double* li = Linv + s.linv + (int64_t)rb * 256 + i * 16;  // Linv[kk][i] at i*16 + kk
                for (int kk = 0; kk < bn; ++kk) acc += li[kk] * fr[(b0 + kk) * NRHS + k];
            }
            xb[tid] = acc;
        }
        __syncthreads();
        if (tid < 16 * NRHS && tid / NRHS < bn) fr[b0 * NRHS + tid] = xb[tid];
        // columns before the block: y_k -= sum_i L[b0+i][k] x_{b0+i}
        for (int k = tid; k < b0; k += NT) {
            double a0 = 0.0, a1 = 0.0;
            const double* lk = P + (int64_t)k * d + b0;
            for (int i = 0; i < bn; ++i) {
                a0 += lk[i] * xb[i * NRHS];
                if (NRHS == 2) a1 += lk[i] * xb[i * NRHS + 1];
            }
            fr[k * NRHS] -= a0;
            if (NRHS == 2) fr[k * NRHS + 1] -= a1;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < ns * NRHS; idx += NT) xs[idx] = fr[idx];
}

__global__ __launch_bounds__(NT) void xgather_kernel(int nrhs, int64_t n_lambda, const int32_t* __restrict__ gptr,
                                                     const XGatherEnt* __restrict__ ents,
                                                     const double* __restrict__ x, const double* __restrict__ c,
                                                     double* __restrict__ q)
{
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n_lambda) return;
    double acc = 0.0;
    for (int32_t e = gptr[g]; e < gptr[g + 1]; ++e) acc += ents[e].sign * x[ents[e].xpos * nrhs];
    q[g] = c ? acc - c[g] : acc;
}

// x[r] = f[xperm[r]]: a concatenated DOF vector into the permuted row order
__global__ __launch_bounds__(NT) void permute_in_kernel(int64_t n, const int32_t* __restrict__ xperm,
                                                        const double* __restrict__ f, double* __restrict__ x)
{
    const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (r < n) x[r] = f[xperm[r]];
}

__global__ __launch_bounds__(NT) void elem_adjoint_kernel(int64_t nelem, const ElemRef* __restrict__ elems,
                                                          const int32_t* __restrict__ epos,
                                                          const double* __restrict__ dk,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ dtheta)
{
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= nelem) return;
    const ElemRef E = elems[e];
    const int32_t* pos = epos + E.pos_off;
    const double* K = dk + E.dk_off;
    double acc = 0.0;
    for (int a = 0; a < E.edofs; ++a) {
        const double ga = x[(int64_t)pos[a] * 2];
        double t = 0.0;
        for (int b = 0; b < E.edofs; ++b) t += K[a * E.edofs + b] * x[(int64_t)pos[b] * 2 + 1];
        acc += ga * t;
    }
    dtheta[e] = -acc;
}

// ---------------------------------------------------------------- SYRK


constexpr int ST = 64;   // output tile edge
constexpr int SK = 16;   // rows of X per LDS stage
constexpr int SP = ST + 2;

// One work-group forms one 64x64 tile (rows ta, columns tb) of the lower
// triangle of F~_i = X_i^T X_i, summing over the supernodes whose RHS range
// meets both column ranges (only their rows of X are non-zero there).
// Wavefront w computes the 32x32 quadrant (w/2, w%2) as 2x2 MFMA blocks.  X
// rows go through LDS 16 at a time, zero outside the range, in a software
// pipeline: the global loads of a 16-row stage are requested two stages
// ahead (two register sets), and the two LDS buffers alternate, so each
// stage needs one barrier.  On diagonal tiles the two column ranges
// coincide and one buffer serves both operands.  A wavefront skips the MFMAs
// whose operands are zero throughout: a 16-column block that misses the
// stage's RHS range, the k-steps past the supernode's last row, and on a
// diagonal tile the quadrant above the diagonal (never stored).  The tests
// are uniform over the wavefront and leave every sum unchanged.
template <typename T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void syrk_kernel(const SyrkTile* __restrict__ tiles,
                                                  const int32_t* __restrict__ lists,
                                                  const DevSN* __restrict__ sns,
                                                  const double* __restrict__ X, T* __restrict__ F)
{
    __shared__ double sa[2][SK][SP];
    __shared__ double sb[2][SK][SP];
    constexpr int U = (SK * ST) / NT;   // staged values per thread and operand
    const SyrkTile t = tiles[blockIdx.x];
    if (t.m == 0) return;  // padding tile of the die-aware order (whole work-group)
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int q = lane >> 4, j = lane & 15;
    const int wi = wv >> 1, wj = wv & 1;
    const int ca0 = t.ta * ST, cb0 = t.tb * ST;
    const bool diag = t.ta == t.tb;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    // stages: 16-row pieces of the listed supernodes, in list order; the
    // fetch cursor (supernode fl, rows fk ..) runs two stages ahead
    int nst = 0;
    for (int l = t.list0; l < t.list1; ++l) nst += (sns[lists[l]].ncols + SK - 1) / SK;
    int fl = t.list0, fk = 0;
    // A wavefront's load u reads one X row of the stage (row wv + 4u, lane =
    // column): a buffer descriptor over that row's RHS range returns zero
    // for the columns outside it, for rows past the supernode (empty range)
    // and for the B operand of a diagonal tile, so every load is issued
    // unconditionally and the compiler waits only for the stage it stages.
    static_assert(ST == 64 && NT == 256, "one X row per wavefront and load");
    // what the multiply of a fetched stage needs: its RHS range [j0, j1) and rows
    struct StageInfo {
        int j0, j1, rows;
    };
    auto fetch = [&](double (&ra)[U], double (&rb)[U], StageInfo& si) {
        const DevSN s = sns[lists[fl]];
        si.j0 = s.j0;
        si.j1 = s.j0 + s.w;
        si.rows = s.ncols - fk < SK ? s.ncols - fk : SK;
        const int la = (ca0 + lane - s.j0) * 8, lb = (cb0 + lane - s.j0) * 8;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = fk + wv + 4 * u;
            const int kin = k < s.ncols ? 1 : 0;
            // rows past the supernode: an empty range at row 0
            const double* xr = X + s.xoff + (int64_t)(k * kin) * s.w;
            const uint32_t nb = (uint32_t)(s.w * kin) * 8u;
            ra[u] = load8_range(xr, nb, la);
            rb[u] = load8_range(xr, diag ? 0u : nb, lb);
        }
        fk += SK;
        if (fk >= s.ncols) {
            ++fl;
            fk = 0;
        }
    };
    auto stage = [&](int st, const double (&ra)[U], const double (&rb)[U]) {
        const int buf = st & 1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + u * NT;
            const int kk = idx / ST, cc = idx - kk * ST;
            sa[buf][kk][cc] = ra[u];
            if (!diag) sb[buf][kk][cc] = rb[u];
        }
        __syncthreads();
    };
    const int ra0 = ca0 + 32 * wi, rb0 = cb0 + 32 * wj;   // first columns of the quadrant's blocks
    const bool upper = diag && wi < wj;                    // quadrant above the diagonal
    auto multiply = [&](int st, const StageInfo& si) {
        const int buf = st & 1;
        const double(*pb)[SP] = diag ? sa[buf] : sb[buf];
        // 16-column blocks of the quadrant that meet the stage's range
        const bool ia0 = !upper && ra0 < si.j1 && ra0 + 16 > si.j0;
        const bool ia1 = !upper && ra0 + 16 < si.j1 && ra0 + 32 > si.j0;
        const bool ib0 = rb0 < si.j1 && rb0 + 16 > si.j0;
        const bool ib1 = rb0 + 16 < si.j1 && rb0 + 32 > si.j0;
        if (!((ia0 || ia1) && (ib0 || ib1))) return;
#pragma unroll
        for (int k4 = 0; k4 < SK / 4; ++k4) {
            if (4 * k4 >= si.rows) break;
            const int kr = 4 * k4 + q;
            const double a0 = sa[buf][kr][32 * wi + j], a1 = sa[buf][kr][32 * wi + 16 + j];
            const double b0 = pb[kr][32 * wj + j], b1 = pb[kr][32 * wj + 16 + j];
            if (ia0 && ib0) acc[0][0] = mfma16(a0, b0, acc[0][0]);
            if (ia0 && ib1) acc[0][1] = mfma16(a0, b1, acc[0][1]);
            if (ia1 && ib0) acc[1][0] = mfma16(a1, b0, acc[1][0]);
            if (ia1 && ib1) acc[1][1] = mfma16(a1, b1, acc[1][1]);
        }
    };
    // two register sets: stage st's values were requested two stages earlier
    double r0a[U], r0b[U], r1a[U], r1b[U];
    StageInfo f0{}, f1{}, cur{};
    if (nst > 0) fetch(r0a, r0b, f0);
    if (nst > 1) fetch(r1a, r1b, f1);
    for (int st = 0; st < nst; st += 2) {
        stage(st, r0a, r0b);
        cur = f0;
        if (st + 2 < nst) fetch(r0a, r0b, f0);
        multiply(st, cur);
        if (st + 1 >= nst) break;
        stage(st + 1, r1a, r1b);
        cur = f1;
        if (st + 3 < nst) fetch(r1a, r1b, f1);
        multiply(st + 1, cur);
    }
    constexpr int64_t V = kRowAlignBytes / sizeof(T);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ca0 + 32 * wi + 16 * a + q + 4 * r;
            if (row >= t.m) continue;
            T* frow = F + t.fbase + packed_row_offset(row, V);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = cb0 + 32 * wj + 16 * b + j;
                if (col <= row) store_f<T>(frow + col, acc[a][b][r]);
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

template <typename T>
constexpr int prec_of()
{
    return sizeof(T) == 8 ? 0 : (sizeof(T) == 4 ? 1 : 2);
}

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

// 16 bytes per lane from a buffer descriptor covering [base, base + nbytes):
// lanes whose 16 bytes fall outside read zero (hardware range check), so the
// base and range can be wavefront-uniform (scalar registers) and one lane
// offset register serves every load.  Descriptor word 3 is the gfx9-family
// raw-buffer format.
template <bool NTL>
__device__ __forceinline__ uint4 load16_range(const void* base, uint32_t nbytes, int lane_off)
{
    __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nbytes, 0x00020000);
    u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, 0, NTL ? 2 : 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// A descriptor over one padded row [base, base + nbytes) and 16-byte loads at
// byte offsets into it: an offset at or past nbytes reads zero.  One
// descriptor serves every chunk of the row (the chunk's position is part of
// the per-lane offset), so the scalar work is per row, not per load.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nbytes, 0x00020000);
}
template <bool NTL>
__device__ __forceinline__ uint4 load16_at(__amdgpu_buffer_rsrc_t r, int off)
{
    u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NTL ? 2 : 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}

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

// One work-group handles an equal share of all stored elements: a short list
// of segments, each a band of rows [r0, r1) of one packed lower triangle.
// Every stored element F[r][c] (c <= r) contributes F[r][c] p[c] to row r (a
// dot product) and, for c < r, F[r][c] p[r] to row c (kept in per-lane
// registers).  A segment writes its partial vector z[0..r1).
// The four wavefronts form two pairs; a pair takes ROWS consecutive rows per
// pass and its two wavefronts split every row's 16-byte column chunks
// round-robin (chunk ch belongs to wavefront ch % 2 of the pair), so each
// lane keeps the column partials of only half the chunks and more rows'
// loads are in flight at once.  Row dots are the sum of the two wavefronts'
// partials, added in a fixed order at the end.  Row padding is zero (F is
// cleared at creation and only c <= r is ever stored) and so is p beyond r1,
// so the inner loop needs no per-element test except keeping the diagonal
// out of the column partials, and that only in the chunks that reach the
// pass's first row.
template <typename T, int NCH, int ROWS, bool NTL>
__global__ __launch_bounds__(NT) void apply_band_kernel(const Band* __restrict__ bands,
                                                        const int32_t* __restrict__ seg_ptr,
                                                        const T* __restrict__ F,
                                                        const double* __restrict__ lam,
                                                        const int32_t* __restrict__ dmap,
                                                        typename Acc<T>::type* __restrict__ z)
{
    using A = typename Acc<T>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int RA = kRowAlignBytes / sizeof(T);   // row granularity of the packed layout
    constexpr int CH = 64 * VEC;          // columns per chunk
    constexpr int CAP = NCH * CH;
    constexpr int NH = (NCH + 1) / 2;     // chunks per wavefront of a pair
    __shared__ A sp[CAP];                 // p = lambda[D_i] (sorted order), zero beyond r1; later partial sums
    __shared__ A srow[2][CAP];            // row-dot partials of the two wavefronts of a pair
    const int tid = threadIdx.x, lane = tid & 63;
    // wavefront-uniform values in scalar registers: row indices, row
    // addresses and loop control then stay out of the vector registers
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int pair = wv >> 1, half = wv & 1;
    for (int seg = seg_ptr[blockIdx.x]; seg < seg_ptr[blockIdx.x + 1]; ++seg) {
    const Band b = bands[seg];
    for (int cidx = tid; cidx < CAP; cidx += NT) sp[cidx] = cidx < b.r1 ? (A)lam[dmap[b.dbase + cidx]] : (A)0;
    __syncthreads();
    A y[NH][VEC];
#pragma unroll
    for (int c2 = 0; c2 < NH; ++c2)
#pragma unroll
        for (int e = 0; e < VEC; ++e) y[c2][e] = (A)0;
    const char* __restrict__ tri = reinterpret_cast<const char*>(F + b.fbase);
    // loads of the ROWS rows from r on; rows at or past r1 read zero (empty range)
    auto issue = [&](int r, uint4 (&raw)[ROWS][NH]) {
        // padded row r + k: bytes [row_start, row_start + len); a row's
        // successor starts len bytes later
        int64_t row_start = packed_row_offset(r, RA) * (int64_t)sizeof(T);
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int len = (int)(RA * ((r + k) / RA + 1) * sizeof(T));
            const int row_bytes = r + k < b.r1 ? len : 0;
            const __amdgpu_buffer_rsrc_t rs = row_rsrc(tri + row_start, (uint32_t)row_bytes);
            row_start += len;
#pragma unroll
            for (int c2 = 0; c2 < NH; ++c2) {
                const int ch = 2 * c2 + half;
                raw[k][c2] = ch < NCH ? load16_at<NTL>(rs, ch * CH * (int)sizeof(T) + lane * 16) : make_uint4(0, 0, 0, 0);
            }
        }
    };
    auto consume = [&](int r, const uint4 (&raw)[ROWS][NH]) {
        int rr[ROWS];
        int rmax = r;
        A pr[ROWS], dot[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            rr[k] = (r + k < b.r1) ? r + k : -1;   // -1: no such row
            rmax = rr[k] > rmax ? rr[k] : rmax;
            pr[k] = rr[k] >= 0 ? sp[rr[k]] : (A)0;
            dot[k] = (A)0;
        }
#pragma unroll
        for (int c2 = 0; c2 < NH; ++c2) {
            const int ch = 2 * c2 + half;
            if (ch >= NCH || ch * CH > rmax) break;  // wavefront-uniform
            const int col = ch * CH + lane * VEC;
            A pc[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) pc[e] = sp[col + e];
            // only a chunk reaching column r can hold a diagonal element of
            // the pass's rows (wavefront-uniform test); the others need no mask
            if ((ch + 1) * CH <= r) {
#pragma unroll
                for (int k = 0; k < ROWS; ++k) {
                    A v[VEC];
                    unpack<T, VEC>(raw[k][c2], v);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        dot[k] += v[e] * pc[e];
                        y[c2][e] += v[e] * pr[k];
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < ROWS; ++k) {
                    A v[VEC];
                    unpack<T, VEC>(raw[k][c2], v);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        dot[k] += v[e] * pc[e];
                        y[c2][e] += (col + e == rr[k] ? (A)0 : v[e]) * pr[k];
                    }
                }
            }
        }
        // lane l holds the dot of row r + l / (64 / ROWS)
        const A tot = rows_wave_sum<ROWS>(dot, lane);
        const int k = lane / (64 / ROWS);
        if ((lane & (64 / ROWS - 1)) == 0 && r + k < b.r1) srow[half][r + k - b.r0] = tot;
    };
    if constexpr (NCH <= 8) {
        // software pipeline: the loads of the pair's next pass are in flight
        // while the current pass is computed (two register sets, used in turn)
        uint4 ra[ROWS][NH], rb[ROWS][NH];
        int r = b.r0 + ROWS * pair;
        if (r < b.r1) issue(r, ra);
        while (r < b.r1) {
            issue(r + 2 * ROWS, rb);
            consume(r, ra);
            r += 2 * ROWS;
            if (r >= b.r1) break;
            issue(r + 2 * ROWS, ra);
            consume(r, rb);
            r += 2 * ROWS;
        }
    } else {
        // long rows: one register set (two would not leave room for a
        // second wavefront per SIMD)
        uint4 ra[ROWS][NH];
        for (int r = b.r0 + ROWS * pair; r < b.r1; r += 2 * ROWS) {
            issue(r, ra);
            consume(r, ra);
        }
    }
    __syncthreads();
    // sp is free now: sum the column partials in a fixed order (pair 0, then pair 1)
    for (int w = 0; w < 4; ++w) {
        const int wp = w >> 1, wh = w & 1;   // pair-major order: waves 0,1 (pair 0) then 2,3 (pair 1)
        if (pair == wp && half == wh) {
#pragma unroll
            for (int c2 = 0; c2 < NH; ++c2)
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int ch = 2 * c2 + half;
                    const int cc = ch * CH + lane * VEC + e;
                    if (ch < NCH && cc < b.r1) sp[cc] = (wp == 0 ? (A)0 : sp[cc]) + y[c2][e];
                }
        }
        __syncthreads();
    }
    for (int cidx = tid; cidx < b.r1; cidx += NT)
        z[b.zoff + cidx] = sp[cidx] + (cidx >= b.r0 ? srow[0][cidx - b.r0] + srow[1][cidx - b.r0] : (A)0);
    __syncthreads();  // sp and srow are reused by the next segment
    }
}

// Column-segmented variant for long rows.  The columns [0, r1) of a band
// are taken in segments of SEGCH chunks (SEGCH * 64 * VEC columns); for each
// segment, the band rows that reach into it are spread over the four
// wavefronts, ROWS consecutive rows per pass, each wavefront reading whole
// row pieces (no pair split), so the per-lane column partials and load
// buffers are bounded by the segment, not by m.  p = lambda[D_i] is held in
// LDS for the band's own rows (`spr`, their row scalars) and for the
// current segment's columns (`spc`, refilled per segment, zero past r1), so
// the LDS a work-group needs is bounded by the segment width and the rows
// of a band, whatever m is.  Row dots add up across segments in `sband`
// (one entry per band row); after a segment its column sums are complete:
// columns left of the band go to z at once, the band's own columns are
// added to `sband`.  Every sum has a fixed order.
// Dynamic LDS: spr[brmax], sband[brmax], spc[SEGW], sseg[SEGW].
template <typename T, int SEGCH, int ROWS, bool NTL>
__global__ __launch_bounds__(NT) void apply_seg_kernel(const Band* __restrict__ bands,
                                                       const int32_t* __restrict__ seg_ptr,
                                                       const T* __restrict__ F,
                                                       const double* __restrict__ lam,
                                                       const int32_t* __restrict__ dmap,
                                                       typename Acc<T>::type* __restrict__ z, int32_t brmax)
{
    using A = typename Acc<T>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int RA = kRowAlignBytes / sizeof(T);
    constexpr int CH = 64 * VEC;          // columns per chunk
    constexpr int SEGW = SEGCH * CH;      // columns per segment
    extern __shared__ double smem_d[];
    A* __restrict__ spc = reinterpret_cast<A*>(smem_d);
    A* __restrict__ sseg = spc + SEGW;
    A* __restrict__ spr = sseg + SEGW;
    A* __restrict__ sband = spr + brmax;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int seg = seg_ptr[blockIdx.x]; seg < seg_ptr[blockIdx.x + 1]; ++seg) {
    const Band b = bands[seg];
    for (int c = tid; c < b.r1 - b.r0; c += NT) {
        spr[c] = (A)lam[dmap[b.dbase + b.r0 + c]];
        sband[c] = (A)0;
    }
    const char* __restrict__ tri = reinterpret_cast<const char*>(F + b.fbase);
    const int nseg = (b.r1 + SEGW - 1) / SEGW;
    for (int cs = 0; cs < nseg; ++cs) {
        const int c0 = cs * SEGW;
        for (int c = tid; c < SEGW; c += NT) spc[c] = c0 + c < b.r1 ? (A)lam[dmap[b.dbase + c0 + c]] : (A)0;
        __syncthreads();
        A y[SEGCH][VEC];
#pragma unroll
        for (int ch = 0; ch < SEGCH; ++ch)
#pragma unroll
            for (int e = 0; e < VEC; ++e) y[ch][e] = (A)0;
        // the ROWS rows from r on, this segment's chunks; rows at or past r1
        // and chunks past a row's end read zero (empty range)
        auto issue = [&](int r, uint4 (&raw)[ROWS][SEGCH]) {
            int64_t row_start = packed_row_offset(r, RA) * (int64_t)sizeof(T);
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                const int len = (int)(RA * ((r + k) / RA + 1) * sizeof(T));
                const int row_bytes = r + k < b.r1 ? len : 0;
                const __amdgpu_buffer_rsrc_t rs = row_rsrc(tri + row_start, (uint32_t)row_bytes);
                row_start += len;
#pragma unroll
                for (int ch = 0; ch < SEGCH; ++ch)
                    raw[k][ch] = load16_at<NTL>(rs, (c0 + ch * CH) * (int)sizeof(T) + lane * 16);
            }
        };
        auto consume = [&](int r, const uint4 (&raw)[ROWS][SEGCH]) {
            int rr[ROWS];
            A pr[ROWS], dot[ROWS];
            int rmax = r;
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                rr[k] = (r + k < b.r1) ? r + k : -1;
                rmax = rr[k] > rmax ? rr[k] : rmax;
                pr[k] = rr[k] >= 0 ? spr[rr[k] - b.r0] : (A)0;
                dot[k] = (A)0;
            }
#pragma unroll
            for (int ch = 0; ch < SEGCH; ++ch) {
                if (c0 + ch * CH > rmax) break;  // wavefront-uniform
                const int col = c0 + ch * CH + lane * VEC;
                A pc[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) pc[e] = spc[ch * CH + lane * VEC + e];
                // only a chunk reaching column r can hold a diagonal element
                // of the pass's rows (wavefront-uniform test)
                if (c0 + (ch + 1) * CH <= r) {
#pragma unroll
                    for (int k = 0; k < ROWS; ++k) {
                        A v[VEC];
                        unpack<T, VEC>(raw[k][ch], v);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            dot[k] += v[e] * pc[e];
                            y[ch][e] += v[e] * pr[k];
                        }
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < ROWS; ++k) {
                        A v[VEC];
                        unpack<T, VEC>(raw[k][ch], v);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            dot[k] += v[e] * pc[e];
                            y[ch][e] += (col + e == rr[k] ? (A)0 : v[e]) * pr[k];
                        }
                    }
                }
            }
            const A tot = rows_wave_sum<ROWS>(dot, lane);
            const int k = lane / (64 / ROWS);
            if ((lane & (64 / ROWS - 1)) == 0 && r + k < b.r1) sband[r + k - b.r0] += tot;
        };
        // band rows reaching into the segment: r >= max(r0, c0)
        const int rs = b.r0 > c0 ? b.r0 : c0;
        uint4 ra[ROWS][SEGCH], rb[ROWS][SEGCH];
        int r = rs + ROWS * wv;
        if (r < b.r1) issue(r, ra);
        while (r < b.r1) {
            issue(r + 4 * ROWS, rb);
            consume(r, ra);
            r += 4 * ROWS;
            if (r >= b.r1) break;
            issue(r + 4 * ROWS, ra);
            consume(r, rb);
            r += 4 * ROWS;
        }
        // column sums of the segment, waves added in a fixed order
        for (int w = 0; w < 4; ++w) {
            if (wv == w) {
#pragma unroll
                for (int ch = 0; ch < SEGCH; ++ch)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int cc = ch * CH + lane * VEC + e;
                        sseg[cc] = (w == 0 ? (A)0 : sseg[cc]) + y[ch][e];
                    }
            }
            __syncthreads();
        }
        const int c1 = c0 + SEGW < b.r1 ? c0 + SEGW : b.r1;
        for (int c = c0 + tid; c < c1; c += NT) {
            if (c < b.r0) z[b.zoff + c] = sseg[c - c0];
            else sband[c - b.r0] += sseg[c - c0];
        }
        __syncthreads();
    }
    for (int c = b.r0 + tid; c < b.r1; c += NT) z[b.zoff + c] = sband[c - b.r0];
    __syncthreads();  // LDS is reused by the next band
    }
}

// Streaming-read probe (a measurement aid, no part of the method): work-group
// g reads bytes [g * region, min((g + 1) * region, bytes)) of buf as FP64
// values with 16-byte non-temporal buffer loads, four per lane in flight,
// and writes their sum to out[g].  It measures the read rate the chip gives
// a kernel that streams contiguous regions per work-group, the access
// pattern of the apply's bands.
__global__ __launch_bounds__(NT) void read_probe_kernel(const char* __restrict__ buf, int64_t bytes, int64_t region,
                                                        double* __restrict__ out)
{
    const int64_t beg = (int64_t)blockIdx.x * region;
    const int64_t len = (bytes - beg) < region ? (bytes - beg) : region;
    const char* base = buf + beg;
    double acc = 0.0;
    constexpr int64_t step = (int64_t)NT * 16 * 4;
    for (int64_t o = 0; o < len; o += step) {
        // the window [o, o + step) through a descriptor that ends at the
        // region's end: loads past it read zero
        const char* w = base + o;
        const uint32_t nb = (uint32_t)((len - o) < step ? (len - o) : step);
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = load16_range<true>(w, nb, (k * NT + (int)threadIdx.x) * 16);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double d[2];
            unpack<double, 2>(v[k], d);
            acc += d[0] + d[1];
        }
    }
    acc = wave_sum(acc);
    __shared__ double part[NT / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// q[g]: the partial sums of every band that holds a term of multiplier g,
// read straight from their positions in the partial vectors, in a fixed
// order (one thread per multiplier; two dependent loads per term).
template <typename A>
__global__ __launch_bounds__(NT) void gather_kernel(int64_t n_lambda, const int32_t* __restrict__ zptr,
                                                    const int64_t* __restrict__ zpos, const A* __restrict__ z,
                                                    double* __restrict__ q)
{
    const int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (g >= n_lambda) return;
    double acc = 0.0;
    for (int32_t k = zptr[g]; k < zptr[g + 1]; ++k) acc += (double)z[zpos[k]];
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

hipError_t launch_diag_inverse(const InvItem* items, int32_t nitems, const DevSN* sns, const double* L,
                               double* Linv, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const int64_t threads = (int64_t)nitems * 16;
    hipLaunchKernelGGL(diag_inverse_kernel, dim3((unsigned)((threads + NT - 1) / NT)), dim3(NT), 0, st, items,
                       nitems, sns, L, Linv);
    return hipGetLastError();
}

hipError_t launch_trsm_level(const TrsmItem* items, int32_t nitems, int32_t waves, int32_t max_ns,
                             const DevSN* sns, const double* L, const double* Linv, const int64_t* rowoff,
                             double* X, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const size_t lds = trsm_lds_bytes(waves, max_ns);
    const void* fn = waves == 4 ? (const void*)trsm_level_kernel<4>
                   : waves == 2 ? (const void*)trsm_level_kernel<2> : (const void*)trsm_level_kernel<1>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int32_t nbmax = (max_ns + 15) / 16;
    if (waves == 4)
        hipLaunchKernelGGL(trsm_level_kernel<4>, dim3(nitems), dim3(256), lds, st, items, nbmax, sns, L, Linv, rowoff, X);
    else if (waves == 2)
        hipLaunchKernelGGL(trsm_level_kernel<2>, dim3(nitems), dim3(128), lds, st, items, nbmax, sns, L, Linv, rowoff, X);
    else
        hipLaunchKernelGGL(trsm_level_kernel<1>, dim3(nitems), dim3(64), lds, st, items, nbmax, sns, L, Linv, rowoff, X);
    return hipGetLastError();
}

hipError_t launch_trsm_bwd_level(const TrsmItem* items, int32_t nitems, int32_t waves, const DevSN* pans,
                                 const double* L, const double* Linv, const int64_t* zrow, const double* X, double* Z,
                                 hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (waves == 4)
        hipLaunchKernelGGL(trsm_bwd_level_kernel<4>, dim3(nitems), dim3(256), 0, st, items, pans, L, Linv, zrow, X, Z);
    else if (waves == 2)
        hipLaunchKernelGGL(trsm_bwd_level_kernel<2>, dim3(nitems), dim3(128), 0, st, items, pans, L, Linv, zrow, X, Z);
    else
        hipLaunchKernelGGL(trsm_bwd_level_kernel<1>, dim3(nitems), dim3(64), 0, st, items, pans, L, Linv, zrow, X, Z);
    return hipGetLastError();
}

hipError_t launch_tri_from_z(int prec, int32_t nsub, int64_t nrows, const int32_t* sub_m, const int32_t* start_rows,
                             const int8_t* signs, const int64_t* zbase, const int64_t* fbase, const double* Z,
                             void* F, hipStream_t st)
{
    if (nrows <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nrows + NT / 64 - 1) / (NT / 64)));
    if (prec == 0)
        hipLaunchKernelGGL(tri_from_z_kernel<double>, grid, dim3(NT), 0, st, nsub, nrows, sub_m, start_rows, signs,
                           zbase, fbase, Z, (double*)F);
    else if (prec == 1)
        hipLaunchKernelGGL(tri_from_z_kernel<float>, grid, dim3(NT), 0, st, nsub, nrows, sub_m, start_rows, signs,
                           zbase, fbase, Z, (float*)F);
    else
        hipLaunchKernelGGL(tri_from_z_kernel<bf16_t>, grid, dim3(NT), 0, st, nsub, nrows, sub_m, start_rows, signs,
                           zbase, fbase, Z, (bf16_t*)F);
    return hipGetLastError();
}

hipError_t launch_scatter_dual(int nrhs, int32_t nsub, const int32_t* sub_rowbase, const int32_t* sub_mbase,
                               const int32_t* start_rows, const int8_t* signs_sorted, const int32_t* dmap_sorted,
                               const double* v0, const double* v1, double* x, int64_t nrows_total, hipStream_t st)
{
    (void)nrows_total;
    if (nsub <= 0) return hipSuccess;
    if (nrhs == 1)
        hipLaunchKernelGGL(scatter_dual_kernel<1>, dim3(nsub), dim3(NT), 0, st, sub_rowbase, sub_mbase, start_rows,
                           signs_sorted, dmap_sorted, v0, v1, x);
    else
        hipLaunchKernelGGL(scatter_dual_kernel<2>, dim3(nsub), dim3(NT), 0, st, sub_rowbase, sub_mbase, start_rows,
                           signs_sorted, dmap_sorted, v0, v1, x);
    return hipGetLastError();
}

hipError_t launch_trsv_forward_level(int nrhs, const int32_t* sn_list, int32_t n, int32_t max_front,
                                     const DevSN* sns, const double* L, const double* Linv,
                                     const int32_t* child_ptr, const int32_t* child_idx, const int32_t* relpos,
                                     double* u, double* x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)max_front * nrhs;
    if (nrhs == 1)
        hipLaunchKernelGGL(trsv_forward_kernel<1>, dim3(n), dim3(NT), lds, st, sn_list, sns, L, Linv, child_ptr,
                           child_idx, relpos, u, x);
    else
        hipLaunchKernelGGL(trsv_forward_kernel<2>, dim3(n), dim3(NT), lds, st, sn_list, sns, L, Linv, child_ptr,
                           child_idx, relpos, u, x);
    return hipGetLastError();
}

hipError_t launch_trsv_backward_level(int nrhs, const int32_t* sn_list, int32_t n, int32_t max_front,
                                      const DevSN* sns, const double* L, const double* Linv, const int32_t* rows,
                                      double* x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)max_front * nrhs;
    if (nrhs == 1)
        hipLaunchKernelGGL(trsv_backward_kernel<1>, dim3(n), dim3(NT), lds, st, sn_list, sns, L, Linv, rows, x);
    else
        hipLaunchKernelGGL(trsv_backward_kernel<2>, dim3(n), dim3(NT), lds, st, sn_list, sns, L, Linv, rows, x);
    return hipGetLastError();
}

hipError_t launch_xgather(int nrhs, int64_t n_lambda, const int32_t* gptr, const XGatherEnt* ents, const double* x,
                          const double* c, double* q, hipStream_t st)
{
    if (n_lambda <= 0) return hipSuccess;
    hipLaunchKernelGGL(xgather_kernel, dim3((unsigned)((n_lambda + NT - 1) / NT)), dim3(NT), 0, st, nrhs, n_lambda,
                       gptr, ents, x, c, q);
    return hipGetLastError();
}

hipError_t launch_permute_in(int64_t n, const int32_t* xperm, const double* f, double* x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_in_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, xperm, f, x);
    return hipGetLastError();
}

hipError_t launch_elem_adjoint(int64_t nelem, const ElemRef* elems, const int32_t* epos, const double* dk,
                               const double* x, double* dtheta, hipStream_t st)
{
    if (nelem <= 0) return hipSuccess;
    hipLaunchKernelGGL(elem_adjoint_kernel, dim3((unsigned)((nelem + NT - 1) / NT)), dim3(NT), 0, st, nelem, elems,
                       epos, dk, x, dtheta);
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
static void apply_launch(const Band* bands, const int32_t* seg_ptr, int32_t ngroups, const T* f, const double* lam,
                         const int32_t* dmap, typename Acc<T>::type* z, hipStream_t st)
{
    // a band keeps NCH * 64 * VEC columns of p and of the row sums in LDS;
    // only instantiate shapes whose capacity stays within 4096 columns
    if constexpr (NCH * 64 * (16 / (int)sizeof(T)) <= 4096)
        hipLaunchKernelGGL((apply_band_kernel<T, NCH, ROWS, NTL>), dim3(ngroups), dim3(NT), 0, st, bands, seg_ptr,
                           f, lam, dmap, z);
}

template <typename T, int ROWS, bool NTL>
static hipError_t apply_dispatch_nch(int nch, const Band* bands, const int32_t* seg_ptr, int32_t ngroups,
                                     const void* F, const double* lam, const int32_t* dmap, void* z, hipStream_t st)
{
    using A = typename Acc<T>::type;
    const T* f = (const T*)F;
    A* zz = (A*)z;
    if (nch * 64 * (16 / (int)sizeof(T)) > 4096) return hipErrorInvalidValue;
    switch (nch) {
    case 1: apply_launch<T, 1, ROWS, NTL>(bands, seg_ptr, ngroups, f, lam, dmap, zz, st); break;
    case 2: apply_launch<T, 2, ROWS, NTL>(bands, seg_ptr, ngroups, f, lam, dmap, zz, st); break;
    case 4: apply_launch<T, 4, ROWS, NTL>(bands, seg_ptr, ngroups, f, lam, dmap, zz, st); break;
    case 8: apply_launch<T, 8, ROWS, NTL>(bands, seg_ptr, ngroups, f, lam, dmap, zz, st); break;
    case 16: apply_launch<T, 16, ROWS, NTL>(bands, seg_ptr, ngroups, f, lam, dmap, zz, st); break;
    case 32: apply_launch<T, 32, ROWS, NTL>(bands, seg_ptr, ngroups, f, lam, dmap, zz, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t apply_dispatch(int nch, int rows, bool ntl, const Band* bands, const int32_t* seg_ptr,
                                 int32_t ngroups, const void* F, const double* lam, const int32_t* dmap, void* z,
                                 hipStream_t st)
{
    if (rows == 2)
        return ntl ? apply_dispatch_nch<T, 2, true>(nch, bands, seg_ptr, ngroups, F, lam, dmap, z, st)
                   : apply_dispatch_nch<T, 2, false>(nch, bands, seg_ptr, ngroups, F, lam, dmap, z, st);
    if (rows == 4)
        return ntl ? apply_dispatch_nch<T, 4, true>(nch, bands, seg_ptr, ngroups, F, lam, dmap, z, st)
                   : apply_dispatch_nch<T, 4, false>(nch, bands, seg_ptr, ngroups, F, lam, dmap, z, st);
    return hipErrorInvalidValue;
}

template <typename T, int SEGCH, int ROWS, bool NTL>
static hipError_t seg_launch(const Band* bands, const int32_t* seg_ptr, int32_t ngroups, const void* F,
                             const double* lam, const int32_t* dmap, void* z, int32_t brmax, hipStream_t st)
{
    using A = typename Acc<T>::type;
    const size_t lds = apply_seg_lds_bytes(prec_of<T>(), SEGCH, brmax);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)apply_seg_kernel<T, SEGCH, ROWS, NTL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((apply_seg_kernel<T, SEGCH, ROWS, NTL>), dim3(ngroups), dim3(NT), lds, st, bands, seg_ptr,
                       (const T*)F, lam, dmap, (A*)z, brmax);
    return hipGetLastError();
}

template <typename T>
static hipError_t seg_dispatch(int segch, int rows, bool ntl, const Band* bands, const int32_t* seg_ptr,
                               int32_t ngroups, const void* F, const double* lam, const int32_t* dmap, void* z,
                               int32_t brmax, hipStream_t st)
{
    // instances: (2, 3 or 4 chunks, 2 or 4 rows) and (8 chunks, 2 rows);
    // 8 chunks with 4 rows would not fit two wavefronts per SIMD
    if (segch == 8)
        return ntl ? seg_launch<T, 8, 2, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
                   : seg_launch<T, 8, 2, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
    if (segch == 2) {
        if (rows == 4)
            return ntl ? seg_launch<T, 2, 4, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
                       : seg_launch<T, 2, 4, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
        return ntl ? seg_launch<T, 2, 2, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
                   : seg_launch<T, 2, 2, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
    }
    if (segch == 3) {
        if (rows == 4)
            return ntl ? seg_launch<T, 3, 4, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
                       : seg_launch<T, 3, 4, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
        return ntl ? seg_launch<T, 3, 2, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
                   : seg_launch<T, 3, 2, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
    }
    if (segch != 4) return hipErrorInvalidValue;
    if (rows == 4)
        return ntl ? seg_launch<T, 4, 4, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
                   : seg_launch<T, 4, 4, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
    return ntl ? seg_launch<T, 4, 2, true>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st)
               : seg_launch<T, 4, 2, false>(bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
}

hipError_t launch_apply_seg(int prec, int segch, int rows, bool ntl, const Band* bands, const int32_t* seg_ptr,
                            int32_t ngroups, const void* F, const double* lam, const int32_t* dmap, void* z,
                            int32_t brmax, hipStream_t st)
{
    if (ngroups <= 0) return hipSuccess;
    if (brmax <= 0 || brmax > kMaxBandRows) return hipErrorInvalidValue;
    if (prec == 0) return seg_dispatch<double>(segch, rows, ntl, bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
    if (prec == 1) return seg_dispatch<float>(segch, rows, ntl, bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
    return seg_dispatch<bf16_t>(segch, rows, ntl, bands, seg_ptr, ngroups, F, lam, dmap, z, brmax, st);
}

hipError_t launch_apply_band(int prec, int nch, int rows, bool ntl, const Band* bands, const int32_t* seg_ptr,
                             int32_t ngroups, const void* F, const double* lam, const int32_t* dmap, void* z,
                             hipStream_t st)
{
    if (ngroups <= 0) return hipSuccess;
    if (prec == 0) return apply_dispatch<double>(nch, rows, ntl, bands, seg_ptr, ngroups, F, lam, dmap, z, st);
    if (prec == 1) return apply_dispatch<float>(nch, rows, ntl, bands, seg_ptr, ngroups, F, lam, dmap, z, st);
    return apply_dispatch<bf16_t>(nch, rows, ntl, bands, seg_ptr, ngroups, F, lam, dmap, z, st);
}

// ---------------------------------------------------------------- static scratch

namespace {
// The apply partial vectors of the allocation-free apply.  Host code never
// passes this name to a kernel (in host code it is a stand-in, not a device
// address): it uses the address static_scratch_address returns.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_addr[device] = p;
    }
    *out = scratch_addr[device];
    return hipSuccess;
}

hipError_t launch_read_probe(const void* buf, int64_t bytes, int64_t region, double* out, hipStream_t st)
{
    if (bytes <= 0) return hipSuccess;
    const int64_t groups = (bytes + region - 1) / region;
    hipLaunchKernelGGL(read_probe_kernel, dim3((unsigned)groups), dim3(NT), 0, st, (const char*)buf, bytes, region, out);
    return hipGetLastError();
}

hipError_t launch_gather(int prec, int64_t n_lambda, const int32_t* zptr, const int64_t* zpos, const void* z,
                         double* q, hipStream_t st)
{
    if (n_lambda <= 0) return hipSuccess;
    dim3 grid((unsigned)((n_lambda + NT - 1) / NT));
    if (prec == 0)
        hipLaunchKernelGGL(gather_kernel<double>, grid, dim3(NT), 0, st, n_lambda, zptr, zpos, (const double*)z, q);
    else
        hipLaunchKernelGGL(gather_kernel<float>, grid, dim3(NT), 0, st, n_lambda, zptr, zpos, (const float*)z, q);
    return hipGetLastError();
}

}  // namespace fetif
