// Dual solver on the device: projected conjugate gradients (paper Alg. 1,
// M = I or lumped), FP64 iterative refinement around a reduced-precision operator, and
// the primal recovery of alpha and u (Sec. II).
#include <cmath>
#include <limits>

#include "context.hpp"

namespace {

struct Work {
    double *r, *w, *y, *p, *q, *rt, *dl, *mz, *mz2;
    double *t, *s;
};

Work work_of(fetiF_ctx c)
{
    const int64_t n = c->n_lambda;
    Work W;
    W.r = c->dVec;
    W.w = c->dVec + n;
    W.y = c->dVec + 2 * n;
    W.p = c->dVec + 3 * n;
    W.q = c->dVec + 4 * n;
    W.rt = c->dVec + 5 * n;
    W.dl = c->dVec + 6 * n;
    W.mz = c->dVec + 7 * n;
    W.mz2 = c->dVec + 8 * n;
    W.t = c->dCvec;
    W.s = c->dCvec + c->ncoarse;
    return W;
}

hipError_t apply_op(fetiF_ctx c, int implicit, const double* x, double* out, hipStream_t st)
{
    fetiF_status s = implicit ? fetiF_apply_implicit(c, x, out, st) : fetiF_apply(c, x, out, st);
    return s == FETIF_OK ? hipSuccess : hipErrorUnknown;
}

// out = P in = in - G (G^T G)^{-1} G^T in
hipError_t project(fetiF_ctx c, const Work& W, const double* in, double* out, hipStream_t st)
{
    hipError_t e;
    if ((e = launch_gt(c->nsub, c->dCoarse, c->dGv, c->dDmap, in, W.t, st)) != hipSuccess) return e;
    if ((e = launch_gemv(c->ncoarse, c->dAinv, W.t, W.s, st)) != hipSuccess) return e;
    return launch_gs(c->n_lambda, 1.0, -1.0, c->dGptr2, c->dGent2, c->dGv, W.s, in, out, st);
}

// y = P M w with M = I (precond 0), the lumped preconditioner (precond 1)
// or the lumped preconditioner with the scaled jump operator (precond 2:
// M = B_D K B_D^T, B_D = A^{-1} B W, A = B W B^T block diagonal)
hipError_t precondition(fetiF_ctx c, const Work& W, int precond, const double* w, double* y, hipStream_t st)
{
    if (!precond) return project(c, W, w, y, st);
    hipError_t e;
    const int64_t n = c->n_lambda;
    if (precond == 1) {
        if ((e = launch_lumped_local(c->nsub, c->lb_nbmax, c->dLump, c->dLbUptr, c->dLbUk, c->dLbSgn, c->dLbKptr,
                                     c->dLbKcol, c->dLbKval, c->dLbMb, c->dDmap, w, c->dLbY, st)) != hipSuccess)
            return e;
        if ((e = launch_lumped_gather(n, c->dLbGptr, c->dLbGpos, c->dLbY, W.mz, st)) != hipSuccess) return e;
        return project(c, W, W.mz, y, st);
    }
    if ((e = launch_block_apply(n, c->dSbOf, c->dSbPos, c->dSbPtr, c->dSbMem, c->dSbOff, c->dSbInv, w, W.mz, st)) !=
        hipSuccess)
        return e;
    if ((e = launch_lumped_local(c->nsub, c->lb_nbmax, c->dLump, c->dLbUptr, c->dLbUk, c->dLbCoef, c->dLbKptr,
                                 c->dLbKcol, c->dLbKval, c->dLbMb, c->dDmap, W.mz, c->dLbY, st)) != hipSuccess)
        return e;
    if ((e = launch_lumped_gather(n, c->dLbGptr, c->dLbGpos, c->dLbY, W.mz2, st)) != hipSuccess) return e;
    if ((e = launch_block_apply(n, c->dSbOf, c->dSbPos, c->dSbPtr, c->dSbMem, c->dSbOff, c->dSbInv, W.mz2, W.mz,
                                st)) != hipSuccess)
        return e;
    return project(c, W, W.mz, y, st);
}

// Weights W = diag(K_bb)^{-1} of the scaled jump operator from the current
// K_bb values (host copy), sign * weight per sorted multiplier, and the
// dense inverses of the diagonal blocks of A = B W B^T (Cholesky of each
// small SPD block, then its inverse), copied to the device.
fetiF_status build_scaled_lumped(fetiF_ctx c)
{
    const int32_t nb = (int32_t)c->hSbPtr.size() - 1;
    std::vector<double> coef((size_t)c->sum_m);
    std::vector<double> A((size_t)c->hSbOff.back(), 0.0);
    for (int32_t i = 0; i < c->nsub; ++i) {
        const SubPlan& P = c->subs[i];
        for (size_t u = 0; u + 1 < P.lb_uptr.size(); ++u) {
            const double kd = c->hLbKval[P.lb_kbase + P.lb_kdiag[u]];
            if (!(kd > 0.0))
                return fail(c, FETIF_ENOTSPD, "subdomain " + std::to_string(i) +
                                                  ": non-positive stiffness diagonal on a multiplier DOF");
            const double wgt = 1.0 / kd;
            for (int32_t e1 = P.lb_uptr[u]; e1 < P.lb_uptr[u + 1]; ++e1) {
                const int32_t k1 = P.lb_uk[e1];
                const double s1 = P.lb_ms[k1];
                coef[(size_t)(P.dbase + k1)] = s1 * wgt;
                const int32_t g1 = P.dual_map[P.sigma[k1]];
                const int32_t b = c->hSbOf[(size_t)g1], sz = c->hSbPtr[(size_t)b + 1] - c->hSbPtr[(size_t)b];
                for (int32_t e2 = P.lb_uptr[u]; e2 < P.lb_uptr[u + 1]; ++e2) {
                    const int32_t k2 = P.lb_uk[e2];
                    const int32_t g2 = P.dual_map[P.sigma[k2]];
                    A[(size_t)(c->hSbOff[(size_t)b] + (int64_t)c->hSbPos[(size_t)g1] * sz + c->hSbPos[(size_t)g2])] +=
                        s1 * P.lb_ms[k2] * wgt;
                }
            }
        }
    }
    // invert every block: Cholesky A = R^T R, then A^{-1} column by column
    std::vector<double> inv(A.size());
    std::vector<double> Rm, x;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t s = c->hSbPtr[(size_t)b + 1] - c->hSbPtr[(size_t)b];
        const double* a = A.data() + c->hSbOff[(size_t)b];
        Rm.assign((size_t)s * s, 0.0);
        for (int32_t j = 0; j < s; ++j) {
            double d = a[j * s + j];
            for (int32_t k = 0; k < j; ++k) d -= Rm[(size_t)(k * s + j)] * Rm[(size_t)(k * s + j)];
            if (!(d > 0.0)) return fail(c, FETIF_ENOTSPD, "a block of B W B^T is not positive definite");
            const double r = std::sqrt(d);
            Rm[(size_t)(j * s + j)] = r;
            for (int32_t t = j + 1; t < s; ++t) {
                double v = a[j * s + t];
                for (int32_t k = 0; k < j; ++k) v -= Rm[(size_t)(k * s + j)] * Rm[(size_t)(k * s + t)];
                Rm[(size_t)(j * s + t)] = v / r;
            }
        }
        double* out = inv.data() + c->hSbOff[(size_t)b];
        x.assign((size_t)s, 0.0);
        for (int32_t col = 0; col < s; ++col) {
            // R^T y = e_col, then R x = y
            for (int32_t t = 0; t < s; ++t) {
                double v = t == col ? 1.0 : 0.0;
                for (int32_t k = 0; k < t; ++k) v -= Rm[(size_t)(k * s + t)] * x[(size_t)k];
                x[(size_t)t] = v / Rm[(size_t)(t * s + t)];
            }
            for (int32_t t = s - 1; t >= 0; --t) {
                double v = x[(size_t)t];
                for (int32_t k = t + 1; k < s; ++k) v -= Rm[(size_t)(t * s + k)] * x[(size_t)k];
                x[(size_t)t] = v / Rm[(size_t)(t * s + t)];
            }
            for (int32_t t = 0; t < s; ++t) out[t * s + col] = x[(size_t)t];
        }
    }
    HIPCHK(c, hipMemcpy(c->dLbCoef, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->dSbInv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
    c->sb_dirty = false;
    return FETIF_OK;
}

// one iteration of Alg. 1 (the loop body), all scalars on the device
hipError_t iteration(fetiF_ctx c, const Work& W, int implicit, int precond, double* lam, hipStream_t st)
{
    hipError_t e;
    const int64_t n = c->n_lambda;
    if ((e = apply_op(c, implicit, W.p, W.q, st)) != hipSuccess) return e;
    if ((e = launch_dot(n, W.p, W.q, nullptr, 1, c->dPart, c->dSc, c->dHist, c->hist_cap, st)) != hipSuccess)
        return e;
    if ((e = launch_update_lr(n, c->dSc, W.p, W.q, lam, W.r, st)) != hipSuccess) return e;
    if ((e = project(c, W, W.r, W.w, st)) != hipSuccess) return e;
    if ((e = precondition(c, W, precond, W.w, W.y, st)) != hipSuccess) return e;  // y = P M w
    if ((e = launch_dot(n, W.w, W.y, W.w, 2, c->dPart, c->dSc, c->dHist, c->hist_cap, st)) != hipSuccess) return e;
    return launch_update_p(n, 1, c->dSc, W.y, W.p, st);
}

hipError_t ensure_hist(fetiF_ctx c, int32_t cap)
{
    if (cap <= c->hist_cap) return hipSuccess;
    if (c->dHist) (void)hipFree(c->dHist);
    if (c->hHist) (void)hipHostFree(c->hHist);
    c->dHist = nullptr;
    c->hHist = nullptr;
    c->hist_cap = 0;
    hipError_t e = hipMalloc((void**)&c->dHist, sizeof(double) * (size_t)cap);
    if (e != hipSuccess) return e;
    e = hipHostMalloc((void**)&c->hHist, sizeof(double) * (size_t)cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    c->hist_cap = cap;
    // captured iterations refer to the old history buffer
    if (c->pcpg_graph) {
        (void)hipGraphExecDestroy(c->pcpg_graph);
        c->pcpg_graph = nullptr;
        c->pcpg_graph_key = -1;
    }
    return hipSuccess;
}

// run `count` iterations, replaying a captured chunk when allowed
hipError_t run_iters(fetiF_ctx c, const Work& W, int implicit, int precond, double* lam, int32_t count,
                     int32_t chunk, bool graph, hipStream_t st)
{
    hipError_t e;
    if (graph && st != nullptr && count >= chunk) {
        const int32_t key = (implicit ? 1 : 0) | (precond << 1) | (chunk << 3);
        const bool reuse = c->pcpg_graph && c->pcpg_graph_key == key && c->pcpg_graph_stream == st &&
                           c->pcpg_lam == lam;
        if (!reuse) {
            if (c->pcpg_graph) {
                (void)hipGraphExecDestroy(c->pcpg_graph);
                c->pcpg_graph = nullptr;
            }
            const bool prof = c->profiling;
            c->profiling = false;  // no event records inside the capture
            if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
                c->profiling = prof;
                return e;
            }
            hipError_t ie = hipSuccess;
            for (int32_t k = 0; k < chunk && ie == hipSuccess; ++k) ie = iteration(c, W, implicit, precond, lam, st);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(st, &g);
            c->profiling = prof;
            if (ie != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return ie;
            }
            if (e != hipSuccess) return e;
            e = hipGraphInstantiate(&c->pcpg_graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
            c->pcpg_graph_key = key;
            c->pcpg_graph_stream = st;
            c->pcpg_lam = lam;
        }
        int32_t done = 0;
        for (; done + chunk <= count; done += chunk)
            if ((e = hipGraphLaunch(c->pcpg_graph, st)) != hipSuccess) return e;
        for (; done < count; ++done)
            if ((e = iteration(c, W, implicit, precond, lam, st)) != hipSuccess) return e;
        return hipSuccess;
    }
    for (int32_t k = 0; k < count; ++k)
        if ((e = iteration(c, W, implicit, precond, lam, st)) != hipSuccess) return e;
    return hipSuccess;
}

// PCPG on P F P lambda = P d from lambda_0 = G (G^T G)^{-1} e (e != NULL)
// or lambda_0 = 0 (e == NULL).  Returns the iterations and ||w_k||/||w_0||.
fetiF_status pcpg_core(fetiF_ctx c, const double* d, const double* e, double* lam, double tol, int32_t maxit,
                       int32_t fixed, int implicit, int precond, int32_t check_every, bool graph, hipStream_t st,
                       int32_t* iters_out, double* rel_out, double* w0_out)
{
    const int64_t n = c->n_lambda;
    const Work W = work_of(c);
    const int32_t cap = std::max(fixed, maxit) + 2;
    HIPCHK(c, ensure_hist(c, cap));
    if (e) {
        HIPCHK(c, launch_gemv(c->ncoarse, c->dAinv, e, W.s, st));
        HIPCHK(c, launch_gs(n, 0.0, 1.0, c->dGptr2, c->dGent2, c->dGv, W.s, nullptr, lam, st));
    } else {
        HIPCHK(c, launch_axpby(n, 0.0, d, 0.0, d, lam, st));
    }
    HIPCHK(c, apply_op(c, implicit, lam, W.q, st));
    HIPCHK(c, launch_axpby(n, 1.0, d, -1.0, W.q, W.r, st));
    HIPCHK(c, project(c, W, W.r, W.w, st));
    HIPCHK(c, precondition(c, W, precond, W.w, W.y, st));
    HIPCHK(c, launch_update_p(n, 0, c->dSc, W.y, W.p, st));
    HIPCHK(c, launch_dot(n, W.w, W.y, W.w, 0, c->dPart, c->dSc, c->dHist, c->hist_cap, st));
    int32_t it = 0;
    double h0 = 0.0, hk = 0.0;
    if (fixed > 0) {
        HIPCHK(c, run_iters(c, W, implicit, precond, lam, fixed, std::max(1, check_every), graph, st));
        it = fixed;
        HIPCHK(c, hipMemcpyAsync(c->hHist, c->dHist, sizeof(double) * (size_t)(it + 1), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        h0 = c->hHist[0];
        hk = c->hHist[it];
    } else {
        HIPCHK(c, hipMemcpyAsync(c->hHist, c->dHist, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        h0 = hk = c->hHist[0];
        const double goal = tol * tol * h0;
        bool done = !(h0 > 0.0) || hk <= goal;
        while (!done && it < maxit) {
            const int32_t chunk = std::min(std::max(1, check_every), maxit - it);
            HIPCHK(c, run_iters(c, W, implicit, precond, lam, chunk, std::max(1, check_every), graph, st));
            HIPCHK(c, hipMemcpyAsync(c->hHist + it + 1, c->dHist + it + 1, sizeof(double) * (size_t)chunk,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            it += chunk;
            hk = c->hHist[it];
            for (int32_t k = it - chunk + 1; k <= it; ++k)
                if (c->hHist[k] <= goal) done = true;
            // a reduced-precision operator can be indefinite on the projected
            // space: stop when w^T y is no longer finite or has grown 1e8-fold
            if (!std::isfinite(hk) || hk > 1e8 * h0) done = true;
        }
    }
    if (iters_out) *iters_out = it;
    if (w0_out) *w0_out = std::isfinite(h0) ? std::sqrt(std::max(0.0, h0)) : std::numeric_limits<double>::quiet_NaN();
    // a residual that is not finite (NaN or Inf in the inputs, or an
    // operator that broke down) is reported as NaN, never as converged
    if (rel_out)
        *rel_out = !(std::isfinite(h0) && std::isfinite(hk)) ? std::numeric_limits<double>::quiet_NaN()
                   : h0 > 0.0                                 ? std::sqrt(std::max(0.0, hk) / h0)
                                                              : 0.0;
    return FETIF_OK;
}

fetiF_status need_coarse(fetiF_ctx c)
{
    if (!c->has_coarse) return fail(c, FETIF_ESTATE, "solver entry points need R_i for every subdomain at create");
    return FETIF_OK;
}

}  // namespace

extern "C" fetiF_status fetiF_coarse_rhs(fetiF_ctx c, const double* f_d, double* e_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (fetiF_status s0 = need_coarse(c)) return s0;
    if (!f_d || !e_d) return fail(c, FETIF_EINVAL, "f or e is NULL");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    HIPCHK(c, launch_rtf(c->nsub, c->dCoarse, c->dR, f_d, e_d, (hipStream_t)stream));
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_precond_values(fetiF_ctx c, int32_t first, int32_t count, const double* const* k_vals)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (fetiF_status s0 = need_coarse(c)) return s0;
    if (first < 0 || count <= 0 || first + count > c->nsub || !k_vals)
        return fail(c, FETIF_EINVAL, "subdomain range out of bounds or k_vals NULL");
    for (int32_t k = 0; k < count; ++k)
        if (!k_vals[k]) return fail(c, FETIF_EINVAL, "k_vals entry is NULL");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    // a factor upload may still copy from the staging of these values
    if (c->upload_pending) {
        HIPCHK(c, hipEventSynchronize(c->upload_done));
        c->upload_pending = false;
    }
    HIPCHK(c, hipDeviceSynchronize());   // the lumped preconditioners may be reading them
    for (int32_t k = 0; k < count; ++k) {
        const SubPlan& P = c->subs[first + k];
        for (size_t e = 0; e < P.lb_ksrc.size(); ++e) c->hLbKval[P.lb_kbase + e] = k_vals[k][P.lb_ksrc[e]];
        c->lb_given[(size_t)(first + k)] = 1;
    }
    const SubPlan& P0 = c->subs[first];
    const SubPlan& P1 = c->subs[first + count - 1];
    const int64_t kb0 = P0.lb_kbase, kb1 = P1.lb_kbase + (int64_t)P1.lb_ksrc.size();
    if (kb1 > kb0)
        HIPCHK(c, hipMemcpy(c->dLbKval + kb0, c->hLbKval + kb0, sizeof(double) * (size_t)(kb1 - kb0),
                            hipMemcpyHostToDevice));
    c->sb_dirty = true;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_pcpg(fetiF_ctx c, const double* d_d, const double* e_d, double* lambda_d,
                                   const fetiF_pcpg_options* opt_in, fetiF_pcpg_result* res, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (fetiF_status s0 = need_coarse(c)) return s0;
    if (!d_d || !e_d || !lambda_d) return fail(c, FETIF_EINVAL, "d, e and lambda are required");
    fetiF_pcpg_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt_in) o = *opt_in;
    if (!(o.tol > 0.0)) o.tol = 1e-9;
    if (o.max_iters <= 0) o.max_iters = 1000;
    if (o.check_every <= 0) o.check_every = 10;
    if (!(o.inner_tol > 0.0)) o.inner_tol = 1e-4;
    if (o.fixed_iters < 0) return fail(c, FETIF_EINVAL, "fixed_iters < 0");
    if (o.precond < 0 || o.precond > 2)
        return fail(c, FETIF_EINVAL, "precond must be 0 (none), 1 (lumped) or 2 (lumped, scaled jump operator)");
    if (o.implicit || o.refine || o.precond) {
        if (fetiF_status s1 = need_factors(c)) return s1;
    }
    if (!o.implicit && !c->assembled) return fail(c, FETIF_ESTATE, "explicit PCPG before assemble");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    if (o.precond == 2 && c->sb_dirty) {
        // the device may still read the previous weights and inverses
        HIPCHK(c, hipStreamSynchronize(st));
        if (fetiF_status s2 = build_scaled_lumped(c)) return s2;
    }
    fetiF_pcpg_result R;
    std::memset(&R, 0, sizeof(R));
    const bool graph = o.use_graph != 0;
    if (!o.refine) {
        fetiF_status s = pcpg_core(c, d_d, e_d, lambda_d, o.tol, o.max_iters, o.fixed_iters, o.implicit,
                                   o.precond, o.check_every, graph, st, &R.iters, &R.rel_residual, &R.w0);
        if (s != FETIF_OK) return s;
    } else {
        // outer FP64 refinement: true projected residual with the implicit
        // FP64 operator, inner PCPG on the correction with the stored F~
        const int64_t n = c->n_lambda;
        const Work W = work_of(c);
        HIPCHK(c, launch_gemv(c->ncoarse, c->dAinv, e_d, W.s, st));
        HIPCHK(c, launch_gs(n, 0.0, 1.0, c->dGptr2, c->dGent2, c->dGv, W.s, nullptr, lambda_d, st));
        // Each inner solve stops at inner_tol, after kInnerMax iterations or
        // on divergence; a correction that does not lower the true residual
        // is taken back and the refinement ends there.
        constexpr int32_t kInnerMax = 2000;
        double w0 = 0.0, wk = 0.0, wprev = 0.0;
        int32_t total = 0;
        for (int32_t outer = 0; outer < 50; ++outer) {
            HIPCHK(c, apply_op(c, 1, lambda_d, W.q, st));
            HIPCHK(c, launch_axpby(n, 1.0, d_d, -1.0, W.q, W.rt, st));
            HIPCHK(c, project(c, W, W.rt, W.w, st));
            HIPCHK(c, launch_dot(n, W.w, W.w, nullptr, 3, c->dPart, c->dSc, nullptr, 0, st));
            double ww = 0.0;
            HIPCHK(c, hipMemcpyAsync(&ww, c->dSc + SC_TMP, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (outer == 0 && !std::isfinite(ww)) {
                w0 = wk = std::numeric_limits<double>::quiet_NaN();
                break;
            }
            wk = std::sqrt(std::max(0.0, ww));
            if (outer == 0) w0 = wk;
            if (outer > 0 && !(wk < wprev)) {
                HIPCHK(c, launch_axpby(n, 1.0, lambda_d, -1.0, W.dl, lambda_d, st));
                wk = wprev;
                break;
            }
            R.outer = outer;
            wprev = wk;
            if (!(w0 > 0.0) || wk <= o.tol * w0 || total >= o.max_iters) break;
            int32_t it = 0;
            fetiF_status s = pcpg_core(c, W.rt, nullptr, W.dl, o.inner_tol, std::min(kInnerMax, o.max_iters - total),
                                       0, 0, o.precond, o.check_every, graph, st, &it, nullptr, nullptr);
            if (s != FETIF_OK) return s;
            total += it;
            HIPCHK(c, launch_axpby(n, 1.0, lambda_d, 1.0, W.dl, lambda_d, st));
        }
        R.iters = total;
        R.w0 = w0;
        R.rel_residual = !std::isfinite(w0) ? std::numeric_limits<double>::quiet_NaN() : w0 > 0.0 ? wk / w0 : 0.0;
    }
    if (res) *res = R;
    return FETIF_OK;
}

extern "C" fetiF_status fetiF_primal(fetiF_ctx c, const double* f_d, const double* d_d, const double* lambda_d,
                                     double* alpha_d, double* u_d, void* stream)
{
    if (!c) return FETIF_EINVAL;
    if (c->sticky) return FETIF_EDEVICE;
    if (fetiF_status s0 = need_coarse(c)) return s0;
    if (fetiF_status s1 = need_factors(c)) return s1;
    if (!f_d || !d_d || !lambda_d || !alpha_d || !u_d) return fail(c, FETIF_EINVAL, "NULL argument");
    DeviceGuard dg(c->device);
    if (!dg.ok) return hip_fail(c, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = c->n_lambda;
    const Work W = work_of(c);
    // alpha = -(G^T G)^{-1} G^T (d - F lambda)
    if (fetiF_apply_implicit(c, lambda_d, W.q, st) != FETIF_OK) return FETIF_EDEVICE;
    HIPCHK(c, launch_axpby(n, 1.0, d_d, -1.0, W.q, W.rt, st));
    HIPCHK(c, launch_gt(c->nsub, c->dCoarse, c->dGv, c->dDmap, W.rt, W.t, st));
    HIPCHK(c, launch_gemv(c->ncoarse, c->dAinv, W.t, W.s, st));
    HIPCHK(c, launch_axpby(c->ncoarse, -1.0, W.s, 0.0, W.s, alpha_d, st));
    // u = K^+ (f - B~^T lambda) + R alpha
    HIPCHK(c, launch_load_primal_rhs(c->nsub, c->dSubRow, c->dSubM, c->dXperm, c->dStartRows, c->dSignsSorted,
                                     c->dDmap, f_d, lambda_d, c->dXv, st));
    HIPCHK(c, solve_all(c, 1, st));
    HIPCHK(c, launch_permute_out(c->total_rows, c->dXperm, c->dXv, u_d, st));
    HIPCHK(c, launch_add_kernel_part(c->nsub, c->dCoarse, c->dR, alpha_d, u_d, st));
    return FETIF_OK;
}
