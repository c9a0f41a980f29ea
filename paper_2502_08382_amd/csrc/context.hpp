// The fetiF context and the helpers shared by the library's host files.
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fetiF.h"
#include "device_types.hpp"
#include "host_sparse.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "solver_kernels.hpp"


namespace fetif {

// message of the last failed create (per host thread)
extern thread_local std::string g_create_error;

template <typename Fn>
void parallel_for(int32_t n, int nthreads, Fn fn)
{
    if (nthreads <= 1 || n <= 1) {
        for (int32_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int32_t> next(0);
    std::vector<std::thread> th;
    int nt = std::min<int>(nthreads, n);
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (;;) {
                int32_t i = next.fetch_add(1);
                if (i >= n) break;
                fn(i);
            }
        });
    for (auto& t : th) t.join();
}

struct SubPlan {
    int32_t n = 0, m = 0, dpn = 1;
    int64_t nnzA = 0;
    Symbolic sym;
    std::vector<int32_t> sigma;   // sorted position -> caller's local multiplier
    std::vector<int32_t> start;   // sorted start rows (permuted DOF of each column)
    std::vector<int32_t> j0, w;   // per supernode
    std::vector<int64_t> xoff;    // per supernode, local
    int64_t nx = 0;
    std::vector<int32_t> b_dof, dual_map;
    std::vector<int8_t> b_sign;
    int32_t nelem = 0, edofs = 0;
    std::vector<int32_t> elem_dofs;
    std::vector<double> dK;
    // global placement
    int64_t lbase = 0, xbase = 0, fbase = 0;
    int32_t snbase = 0, rowbase = 0, dbase = 0, band0 = 0, nband = 0;
    int32_t inv0 = 0, ninv = 0;
    int32_t nk = 0;              // kernel dimension (0: none given)
    std::vector<double> R;       // n x nk row-major
    int32_t koff = 0;            // first coarse unknown
    // lumped preconditioner B~ K_reg B~^T: boundary DOFs (those B~ touches),
    // per sorted multiplier its boundary index and sign, the multipliers on
    // each boundary DOF, the K_reg entries among boundary DOFs (CSR over
    // boundary indices; lb_ksrc = position in the caller's value array)
    std::vector<int32_t> lb_dofs, lb_mb, lb_uptr, lb_uk, lb_kptr, lb_kcol;
    std::vector<int32_t> lb_kdiag;   // per boundary DOF: position of its diagonal entry among the K_bb entries
    int64_t lb_kbase = 0;        // first K_bb entry of this subdomain (global)
    std::vector<int8_t> lb_ms;
    std::vector<int64_t> lb_ksrc;
    std::string err;
};

}  // namespace fetif

using namespace fetif;

struct fetiF_ctx_s {
    int device = 0;
    int64_t n_lambda = 0;
    int32_t nsub = 0;
    fetiF_options opt{};
    int prec = 0;
    int nthreads = 1;
    std::vector<SubPlan> subs;
    // schedules
    // TRSM schedule (per panel level: wavefronts per work-group, widest panel)
    int32_t trsm_levels = 0;
    std::vector<int32_t> level_waves, level_maxns;
    std::vector<DevSN> hSN;          // host copy of the supernode table (TRSM re-planning)
    std::vector<int64_t> hRowOff;    // per global row slot: X offset minus its range start
    int32_t ninv = 0;
    int64_t total_linv = 0;
    // batched solves with L: levels of all supernodes, tree tables
    std::vector<std::vector<int32_t>> solve_levels;
    std::vector<int32_t> solve_maxfront;
    std::vector<int64_t> solve_off;
    int64_t total_u = 0;
    int64_t nelem_total = 0;
    bool has_elems = false;
    std::vector<int64_t> level_off;   // TRSM items of group g, level L: [g * levels + L, .. + 1)
    std::vector<int32_t> grp_first;   // assembly group g = subdomains [grp_first[g], grp_first[g+1])
    std::vector<int64_t> syrk_off;    // SYRK tiles of group g: [syrk_off[g], syrk_off[g+1])
    int32_t apply_nch = 1;
    int32_t nbands = 0;
    int32_t nsyrk = 0;
    int64_t total_L = 0, total_X = 0, total_F = 0, total_z = 0, total_rows = 0, sum_m = 0;
    double trsm_flops = 0, syrk_flops = 0, factor_flops = 0;
    // device buffers
    double* dL = nullptr;
    double* dX = nullptr;
    double* dLinv = nullptr;
    InvItem* dInv = nullptr;
    int32_t* dSolveSn = nullptr;    // supernode ids per solve level
    int32_t* dChildPtr = nullptr;
    int32_t* dChildIdx = nullptr;
    int32_t* dRelpos = nullptr;
    double* dU = nullptr;           // update vectors (2 rhs)
    double* dXv = nullptr;          // solve vectors (2 rhs, permuted rows)
    int32_t* dSubRow = nullptr;     // nsub+1 row bases
    int32_t* dSubM = nullptr;       // nsub+1 multiplier bases
    int32_t* dStartRows = nullptr;  // sorted start rows per subdomain
    int8_t* dSignsSorted = nullptr;
    int32_t* dXGptr = nullptr;
    XGatherEnt* dXGent = nullptr;
    int32_t* dXperm = nullptr;      // x row -> position in the concatenated DOF vector
    ElemRef* dElems = nullptr;
    int32_t* dEpos = nullptr;
    double* dDK = nullptr;
    void* dF = nullptr;
    unsigned long long* dDbg = nullptr;   // first non-finite index of a debug scan (option debug_checks)
    void* dZ = nullptr;
    void* dScratch = nullptr;  // device address of the static scratch (fetiF_apply_static)
    // host-vector application (fetiF_apply_host): host copies of the sorted
    // dual map and of the gather map, and buffers made on first use
    std::vector<int32_t> hDmap;       // sum m_i: global multiplier of sorted local row (dDmap on the host)
    std::vector<int32_t> hZptr;       // gather map of the current apply plan (dZptr, dZpos on the host)
    std::vector<int64_t> hZpos;
    int32_t* dDmapId = nullptr;       // identity map 0 .. sum m_i - 1
    double* dHostVec = nullptr;       // device: lambda (n_lambda) | q (n_lambda) | p (sum m_i)
    double* hPin = nullptr;           // pinned: lambda | q | p (as above), then the partials
    size_t hPinBytes = 0;
    DevSN* dSN = nullptr;
    int32_t* dRows = nullptr;
    DevSN* dTSN = nullptr;     // TRSM column panels
    int64_t* dTRowOff = nullptr; // X offset (minus range start) of their below rows
    XRow* dXRows = nullptr;
    RhsUnit* dUnits = nullptr;
    TrsmItem* dItems = nullptr;
    SyrkTile* dTiles = nullptr;
    int32_t* dLists = nullptr;
    Band* dBands = nullptr;
    int32_t* dSegPtr = nullptr;
    int32_t ngroups = 0;
    int32_t apply_brmax = 0;     // most rows of an apply band
    int32_t max_m = 0;           // largest local multiplier count
    int32_t* dZptr = nullptr;    // gather: multiplier g sums z[dZpos[dZptr[g] .. dZptr[g+1])]
    int64_t* dZpos = nullptr;
    int32_t* dDmap = nullptr;
    double* hStage = nullptr;  // pinned staging of factor values
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    std::vector<void*> allocations;
    std::vector<void*> apply_allocs;  // buffers of the current apply plan
    std::vector<void*> trsm_allocs;   // buffers of the current TRSM plan
    // TRSM path of the assembly (assembly_path 1): backward solve Z = L^{-T} X
    // over column panels of every supernode, then F~ = B~ P^T Z
    int32_t assembly_path = 0;
    std::vector<void*> bwd_allocs;    // Z, its panel tables and the F gather tables
    double* dZfull = nullptr;         // sum n_i m_i, row-major per subdomain
    DevSN* dBPan = nullptr;
    int64_t* dBZrow = nullptr;
    TrsmItem* dBItems = nullptr;
    int64_t* dZbase = nullptr;        // per subdomain: offset of Z_i
    int64_t* dFbase = nullptr;        // per subdomain: offset of F~_i
    std::vector<int64_t> blevel_off;  // backward items of panel level L: [blevel_off[L], blevel_off[L + 1])
    int64_t total_zfull = 0;
    double trsm_bwd_flops = 0;
    // phase timing
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    bool profiling = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[FETIF_NPHASES] = {0};
    int64_t prof_cnt[FETIF_NPHASES] = {0};
    // coarse space and solver (present when every subdomain gave R_i)
    bool has_coarse = false;
    int32_t ncoarse = 0;
    CoarseSub* dCoarse = nullptr;
    double* dGv = nullptr;
    int32_t* dGptr2 = nullptr;
    GEnt* dGent2 = nullptr;
    double* dAinv = nullptr;   // (G^T G)^{-1}, dense ncoarse x ncoarse
    double* dR = nullptr;      // concatenated R_i (sum n_i x nk_i)
    double* dVec = nullptr;    // solver work vectors, 7 x n_lambda
    double* dCvec = nullptr;   // 3 x ncoarse
    // lumped preconditioner (device tables; K_bb values refreshed by every factor upload)
    LumpSub* dLump = nullptr;
    int32_t *dLbUptr = nullptr, *dLbUk = nullptr, *dLbKptr = nullptr, *dLbKcol = nullptr, *dLbMb = nullptr;
    int32_t *dLbGptr = nullptr, *dLbGpos = nullptr;
    double* dLbSgn = nullptr;      // sign of each sorted multiplier (the lumped M)
    // scaled lumped preconditioner (precond 2): M = A^{-1} (sum_i D_i^T B~_i W_i K_bb,i W_i B~_i^T D_i) A^{-1},
    // A = sum_i D_i^T B~_i W_i B~_i^T D_i, W_i = diag(K_bb,i)^{-1}; A is block diagonal over the
    // groups of multipliers that share a (subdomain, DOF): dense inverses of those blocks
    double* dLbCoef = nullptr;     // sign * weight of each sorted multiplier
    int32_t *dSbOf = nullptr, *dSbPos = nullptr, *dSbPtr = nullptr, *dSbMem = nullptr;
    int64_t* dSbOff = nullptr;
    double* dSbInv = nullptr;
    std::vector<int32_t> hSbOf, hSbPos, hSbPtr, hSbMem;
    std::vector<int64_t> hSbOff;
    std::vector<char> lb_given;    // per subdomain: K_bb values from fetiF_precond_values
    bool sb_dirty = true;          // K_bb values changed since the weights and A^{-1} were formed
    double* dLbKval = nullptr;
    double* dLbY = nullptr;    // sum m_i partial results
    double* hLbKval = nullptr; // pinned staging of the K_bb values
    int64_t lb_nk = 0;         // K_bb entries over all subdomains
    int32_t lb_nbmax = 0;
    double* dPart = nullptr;   // 2 x dot_parts(n_lambda)
    double* dSc = nullptr;     // SC_COUNT scalars
    double* dHist = nullptr;   // ||w_k||^2 history
    double* hHist = nullptr;   // pinned copy
    int32_t hist_cap = 0;
    // captured solver iterations (rebuilt when the apply plan changes)
    hipGraphExec_t pcpg_graph = nullptr;
    hipStream_t pcpg_graph_stream = nullptr;
    int32_t pcpg_graph_key = -1;
    const double* pcpg_lam = nullptr;
    // state
    std::vector<uint8_t> uploaded;
    int32_t n_uploaded = 0;
    bool assembled = false;
    bool sticky = false;
    std::string last_error;
};

namespace fetif {

inline fetiF_status fail(fetiF_ctx c, fetiF_status st, const std::string& msg)
{
    if (c) c->last_error = msg;
    else g_create_error = msg;
    return st;
}

inline fetiF_status hip_fail(fetiF_ctx c, hipError_t e, const char* what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (c) {
        c->sticky = true;
        c->last_error = msg;
    } else {
        g_create_error = msg;
    }
    return FETIF_EDEVICE;
}

// Event pair around one device phase when profiling is on.
struct PhaseTimer {
    fetiF_ctx c;
    hipStream_t st;
    int phase;
    hipEvent_t b = nullptr;
    hipError_t err = hipSuccess;
    hipEvent_t get()
    {
        if (!c->ev_pool.empty()) {
            hipEvent_t e = c->ev_pool.back();
            c->ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        err = hipEventCreate(&e);
        return e;
    }
    PhaseTimer(fetiF_ctx c_, hipStream_t s_, int ph) : c(c_), st(s_), phase(ph)
    {
        if (!c->profiling) return;
        hipEvent_t a = get();
        b = get();
        if (err == hipSuccess) err = hipEventRecord(a, st);
        c->recs.push_back({phase, a, b});
    }
    hipError_t stop()
    {
        if (!c->profiling || !b) return err;
        if (err == hipSuccess) err = hipEventRecord(b, st);
        return err;
    }
};

#define HIPCHK(ctx, call)                                         \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);  \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename T>
hipError_t dalloc(fetiF_ctx c, T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * count);
    if (e == hipSuccess) {
        c->allocations.push_back(q);
        *p = (T*)q;
    }
    return e;
}

template <typename T>
hipError_t upload(T* d, const std::vector<T>& h)
{
    if (h.empty()) return hipSuccess;
    return hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
}


// Orders `st` after the last factor copy (its event), so a copy made on
// another stream is complete before the factors are read; skipped while
// `st` is being captured into a graph (the caller orders captured work).
inline hipError_t order_after_upload(fetiF_ctx c, hipStream_t st)
{
    if (!c->upload_pending) return hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    return hipStreamWaitEvent(st, c->upload_done, 0);
}

// batched forward + backward solves with every L_i on c->dXv (context.cpp)
hipError_t solve_all(fetiF_ctx c, int nrhs, hipStream_t st);
// FETIF_ESTATE unless every subdomain has been factored
fetiF_status need_factors(fetiF_ctx c);

}  // namespace fetif
