// The augmented topological level-set loop (Sec. 3.2-3.4, 3.6, 3.8; Fig. 6-7):
// Pareto tracing of minimum volume under a hard compliance constraint (and
// optionally stress and eigenvalue constraints), as a host state machine over
// the library's device steps (solve, energy fields, eigenpair, combined level
// set, casting projection, ranking).  Every per-element step
// runs on the GPU; the host keeps the scalars (J, g, mu, gamma, v, dv).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "afd_internal.h"

namespace {

struct Dev {
    double* rho = nullptr;      // n_elem
    uint8_t* solid = nullptr;   // n_elem, topology to solve
    double* S = nullptr;        // energy fields (see the layout in afd_levelset_run)
    double* raw = nullptr;      // n_elem, T_L of this solve
    double* cur = nullptr;      // n_elem, T_L after damping
    double* src = nullptr;      // n_elem, the level set the solved topology was extracted from
    double* best = nullptr;     // n_elem, level set of the last converged feasible design
    double* cast = nullptr;     // n_elem, projected field
    int32_t* dist = nullptr;    // n_elem, parting-plane distance
    double* F = nullptr;        // nload x n_dof
    double* UL = nullptr;       // nload x n_dof displacements, then (stress) nload x n_dof adjoint fields
    double* B = nullptr;        // nload x n_dof adjoint right-hand sides (stress)
    double* J = nullptr;        // nload
    double* Phi = nullptr;      // n_dof, lowest mode (eigenvalue constraint)
    double* SL = nullptr;       // n_elem, its eigenvalue field
    double* XB = nullptr;       // 4 x n_dof, the eigen-solver's last Ritz block (start of the next one)
    double* PhiB = nullptr;     // n_dof, buckling mode (buckling constraint)
    double* SP = nullptr;       // n_elem, its load-factor field
    double* XBB = nullptr;      // 4 x n_dof, the buckling solver's last Ritz block
    void release() {
        for (void* p : {(void*)rho, (void*)solid, (void*)S, (void*)raw, (void*)cur, (void*)src, (void*)best,
                        (void*)cast, (void*)dist, (void*)F, (void*)UL, (void*)B, (void*)J, (void*)Phi, (void*)SL,
                        (void*)XB, (void*)PhiB, (void*)SP, (void*)XBB})
            if (p) (void)afd::dev_free(p);
    }
};

template <typename T>
int alloc(T** p, size_t n) {
    if (afd::dev_malloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        afd::set_error("levelset: out of device memory");
        return AFD_E_OOM;
    }
    return AFD_OK;
}

// Eq. 3.11 and Eq. 3.12 as printed, from the values before the update
// (k = 0: no previous constraint value, gamma kept)
void al_update(double& mu, double& gamma, double g, double g_old, int k, double varsigma, double eta) {
    const double mu_next = std::max(mu + gamma * g, 0.0);
    double gamma_next = gamma;
    if (k > 0 && !(std::min(g, 0.0) <= varsigma * std::min(g_old, 0.0)))
        gamma_next = std::max(eta * gamma, (double)k * (double)k);
    mu = mu_next;
    gamma = gamma_next;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" int afd_levelset_run(afd_mesh* m, const afd_levelset_opts* o, int32_t nload, const double* F,
                                uint8_t* solid_out, afd_levelset_record* hist, int32_t hist_cap, int32_t* n_hist,
                                uint8_t* topo_hist) {
    using namespace afd;
    if (!m || !o || !F || !solid_out || !hist || hist_cap < 1 || !n_hist || nload < 1 || nload > 4) {
        set_error("levelset: bad argument (nload 1..4, non-null F, solid, hist, n_hist)");
        return AFD_E_INVALID_ARG;
    }
    *n_hist = 0;
    if (!(o->alpha_J >= 1.0) || !(o->dv0 > 0.0 && o->dv0 < 1.0) || !(o->dv_min > 0.0) || !(o->mu0 >= 0.0) ||
        !(o->gamma0 > 0.0) || !(o->varsigma > 0.0 && o->varsigma < 1.0) || !(o->eta > 0.0) ||
        !(o->conv_tol > 0.0) || o->max_fp < 2 || o->max_fea < 1 || !(o->void_scale > 0.0 && o->void_scale <= 1.0) ||
        o->cast_axis < -1 || o->cast_axis > 2) {
        set_error("levelset: bad options (alpha_J >= 1, 0 < dv0 < 1, dv_min > 0, gamma0 > 0, 0 < varsigma < 1, "
                  "eta > 0, conv_tol > 0, max_fp >= 2, max_fea >= 1, 0 < void_scale <= 1, cast_axis -1..2)");
        return AFD_E_INVALID_ARG;
    }
    int64_t ne = 0, nn = 0, nd = 0, nc = 0;
    AFD_TRY(afd_mesh_sizes(m, &ne, &nn, &nd, &nc));
    const afd_mesh_desc& d = mesh_desc(m);
    const int32_t dims[3] = {d.nx, d.ny, d.nz};
    if (o->cast_axis >= 0 && (o->cast_parting < 0 || o->cast_parting > dims[o->cast_axis])) {
        set_error("levelset: cast_parting outside 0..dims[cast_axis]");
        return AFD_E_INVALID_ARG;
    }
    afd_context* ctx = mesh_context(m);
    hipStream_t s = context_stream(ctx);
    {
        // the loads must be finite and vanish on fixed DOFs (as afd_solve checks host loads)
        std::vector<uint8_t> mask(nd);
        AFD_TRY(mesh_dof_mask(m, mask.data()));
        for (int r = 0; r < nload; ++r)
            for (int64_t i = 0; i < nd; ++i) {
                const double f = F[r * nd + i];
                if (!std::isfinite(f) || (mask[i] && f != 0.0)) {
                    set_error("levelset: F must be finite and zero on fixed DOFs");
                    return AFD_E_INVALID_ARG;
                }
            }
    }
    const bool stress = o->alpha_sigma > 0.0;
    if (stress && (nload > 2 || !(o->pnorm_p >= 2.0))) {
        set_error("levelset: the stress constraint needs nload <= 2 and pnorm_p >= 2");
        return AFD_E_INVALID_ARG;
    }
    const bool eigen = o->alpha_lambda > 0.0;
    if (eigen && !(o->alpha_lambda <= 1.0 && o->modal_tol > 0.0)) {
        set_error("levelset: the eigenvalue constraint needs 0 < alpha_lambda <= 1 and modal_tol > 0");
        return AFD_E_INVALID_ARG;
    }
    const bool buck = o->alpha_P > 0.0;
    if (buck && !(o->alpha_P <= 1.0 && o->modal_tol > 0.0)) {
        set_error("levelset: the buckling constraint needs 0 < alpha_P <= 1 and modal_tol > 0");
        return AFD_E_INVALID_ARG;
    }
    // energy fields: without the stress constraint the nload strain-energy
    // fields; with it the afd_sensitivity layout of [U_0..U_n-1, L_0..L_n-1]
    // with the pairs (r, n + r): n strain energies, n adjoint self energies
    // (unused), n mutual energies
    const int nfields = stress ? 3 * nload : nload;
    Dev dv;
    auto fail = [&](int rc) {
        (void)hipStreamSynchronize(s);
        dv.release();
        return rc;
    };
    int rc = AFD_OK;
    if ((rc = alloc(&dv.rho, ne)) || (rc = alloc(&dv.solid, ne)) || (rc = alloc(&dv.S, (size_t)nfields * ne)) ||
        (rc = alloc(&dv.raw, ne)) || (rc = alloc(&dv.cur, ne)) || (rc = alloc(&dv.src, ne)) ||
        (rc = alloc(&dv.best, ne)) || (rc = alloc(&dv.cast, ne)) || (rc = alloc(&dv.dist, ne)) ||
        (rc = alloc(&dv.F, (size_t)nload * nd)) || (rc = alloc(&dv.UL, (size_t)(stress ? 2 : 1) * nload * nd)) ||
        (stress && (rc = alloc(&dv.B, (size_t)nload * nd))) || (rc = alloc(&dv.J, nload)) ||
        (eigen && ((rc = alloc(&dv.Phi, nd)) || (rc = alloc(&dv.SL, ne)) || (rc = alloc(&dv.XB, 4 * nd)))) ||
        (buck && ((rc = alloc(&dv.PhiB, nd)) || (rc = alloc(&dv.SP, ne)) || (rc = alloc(&dv.XBB, 4 * nd)))))
        return fail(rc);
    auto copy = [&](void* dst, const void* src_, size_t bytes, hipMemcpyKind kind) -> int {
        if (hipMemcpyAsync(dst, src_, bytes, kind, s) != hipSuccess) {
            set_error("levelset: copy failed");
            return AFD_E_HIP;
        }
        return AFD_OK;
    };
    if ((rc = copy(dv.F, F, (size_t)nload * nd * sizeof(double), hipMemcpyHostToDevice))) return fail(rc);
    double* Lam = dv.UL + (size_t)nload * nd;
    // topology extraction at volume fraction v from a level-set field, which
    // becomes the source of the next solve's topology
    auto extract = [&](const double* fld, double v) -> int {
        if (o->damping && fld != dv.src) AFD_TRY(copy(dv.src, fld, ne * sizeof(double), hipMemcpyDeviceToDevice));
        if (o->cast_axis >= 0) {
            AFD_TRY(afd_casting(ctx, dims, fld, o->cast_axis, o->cast_parting, dv.cast, dv.dist));
            return afd_threshold(ctx, dv.cast, dv.dist, ne, v, dv.solid, nullptr, nullptr);
        }
        return afd_threshold(ctx, fld, nullptr, ne, v, dv.solid, nullptr, nullptr);
    };
    // the first topology: the full domain
    std::vector<uint8_t> solid_h(ne, 1), best_h(ne, 1);
    if ((rc = copy(dv.solid, solid_h.data(), ne, hipMemcpyHostToDevice))) return fail(rc);
    double mu = o->mu0, gamma = o->gamma0, mu_s = o->mu0, gamma_s = o->gamma0, step = o->dv0, v = 1.0;
    double mu_l = o->mu0, gamma_l = o->gamma0, mu_p = o->mu0, gamma_p = o->gamma0;
    double J0 = 0.0, S0 = 0.0, L0 = 0.0, P0 = 0.0, g_prev = 0.0, gs_prev = 0.0, gl_prev = 0.0, gp_prev = 0.0;
    double J_prev_same = -1.0, v_best = 1.0;  // -1: no previous solve at this target
    int fp = 0;
    bool have_src = false;
    std::vector<afd_solve_stats> st(nload), st2(nload);
    EigenBlock eig_block, buck_block;  // each eigen-solve starts from the previous topology's Ritz block
    eig_block.X = dv.XB;
    buck_block.X = dv.XBB;
    std::vector<double> Jh(nload);
    std::vector<int32_t> pairs(2 * nload);
    for (int r = 0; r < nload; ++r) pairs[2 * r] = r, pairs[2 * r + 1] = nload + r;
    const int kmax = std::min(o->max_fea, hist_cap);
    for (int k = 0; k < kmax; ++k) {
        const double t0 = now_s();
        // step 2: the solves over the current topology (warm-started)
        if ((rc = launch_density(ne, dv.solid, o->void_scale, dv.rho, s))) return fail(rc);
        if ((rc = afd_mesh_set_scale(m, dv.rho, ne, AFD_MEM_DEVICE))) return fail(rc);
        afd_solve_opts so = o->solve;
        so.mem_kind = AFD_MEM_DEVICE;
        so.pairs = nullptr;
        so.npairs = 0;
        so.x0 = k > 0 ? dv.UL : nullptr;
        if ((rc = afd_solve(m, &so, nload, dv.F, dv.UL, dv.J, stress ? nullptr : dv.S, st.data()))) return fail(rc);
        double Sp = 0.0;
        if (stress) {
            // the stress p-norm, its adjoint right-hand sides and adjoint solves
            if ((rc = afd_stress_pnorm(m, nload, dv.UL, o->pnorm_p, nullptr, &Sp, dv.B))) return fail(rc);
            so.x0 = k > 0 ? Lam : nullptr;
            if ((rc = afd_solve(m, &so, nload, dv.B, Lam, nullptr, nullptr, st2.data()))) return fail(rc);
            if ((rc = afd_sensitivity(m, 2 * nload, dv.UL, nload, pairs.data(), dv.S))) return fail(rc);
        }
        double lam = 0.0;
        int modal_cg = 0;
        if (eigen) {
            // the lowest eigenpair of the topology and its field (Eq. 3.4), the
            // subspace iteration started from the previous topology's block
            afd_solve_opts mo = o->solve;
            mo.mem_kind = AFD_MEM_DEVICE;
            mo.pairs = nullptr;
            mo.npairs = 0;
            mo.x0 = nullptr;
            afd_modal_stats ms{};
            if ((rc = modal_with_block(m, &mo, 1, o->modal_tol, 200, &lam, dv.Phi, dv.SL, &ms, &eig_block)))
                return fail(rc);
            modal_cg = ms.cg_iterations;
        }
        double Pb = 0.0;
        if (buck) {
            // the smallest buckling load factor of load case 0 and its field (Eq. 3.5)
            afd_solve_opts bo = o->solve;
            bo.mem_kind = AFD_MEM_DEVICE;
            bo.pairs = nullptr;
            bo.npairs = 0;
            bo.x0 = nullptr;
            afd_modal_stats bs{};
            if ((rc = buckling_with_block(m, dv.UL, &bo, 1, o->modal_tol, 200, &Pb, dv.PhiB, dv.SP, &bs,
                                          &buck_block)))
                return fail(rc);
            modal_cg += bs.cg_iterations;
        }
        if ((rc = copy(Jh.data(), dv.J, nload * sizeof(double), hipMemcpyDeviceToHost)) ||
            (rc = copy(solid_h.data(), dv.solid, ne, hipMemcpyDeviceToHost)))
            return fail(rc);
        if (hipStreamSynchronize(s) != hipSuccess) {
            set_error("levelset: stream sync failed");
            return fail(AFD_E_HIP);
        }
        const double t1 = now_s();
        double J = 0.0;
        int iters = 0;
        for (int r = 0; r < nload; ++r) {
            J += Jh[r];
            iters += st[r].iterations + (stress ? st2[r].iterations : 0);
        }
        iters += modal_cg;
        int nsolid = 0;
        for (int64_t e = 0; e < ne; ++e) nsolid += solid_h[e];
        if (topo_hist) memcpy(topo_hist + (size_t)k * ne, solid_h.data(), ne);
        // step 3: constraint values and the multiplier / penalty updates
        if (k == 0) J0 = J, S0 = Sp, L0 = lam, P0 = Pb;
        const double g = J / (o->alpha_J * J0) - 1.0;
        al_update(mu, gamma, g, g_prev, k, o->varsigma, o->eta);
        g_prev = g;
        double g_s = 0.0;
        if (stress) {
            g_s = Sp / (o->alpha_sigma * S0) - 1.0;
            al_update(mu_s, gamma_s, g_s, gs_prev, k, o->varsigma, o->eta);
            gs_prev = g_s;
        }
        double g_l = 0.0;
        if (eigen) {
            g_l = 1.0 - lam / (o->alpha_lambda * L0);
            al_update(mu_l, gamma_l, g_l, gl_prev, k, o->varsigma, o->eta);
            gl_prev = g_l;
        }
        double g_p = 0.0;
        if (buck) {
            g_p = 1.0 - Pb / (o->alpha_P * P0);
            al_update(mu_p, gamma_p, g_p, gp_prev, k, o->varsigma, o->eta);
            gp_prev = g_p;
        }
        ++fp;
        const bool converged = J_prev_same >= 0.0 && std::fabs(J - J_prev_same) < o->conv_tol * J_prev_same;
        int event;
        if (g > 0.0 || g_s > 0.0 || (g_l > 0.0 && !o->lambda_soft) || (g_p > 0.0 && !o->P_soft))
            event = AFD_LS_VIOLATED;  // step 4: a hard constraint violated
        else if (k == 0 || converged) event = AFD_LS_CONVERGED;  // step 7
        else if (fp >= o->max_fp) event = AFD_LS_DIVERGED;
        else event = AFD_LS_FIXED_POINT;
        const double v_solved = v;
        bool more = true;
        if (event == AFD_LS_VIOLATED || event == AFD_LS_DIVERGED) {
            // step 9: back to the last converged feasible design, half the step
            step *= 0.5;
            if (step < o->dv_min || v_best - step <= 0.0) {
                event = AFD_LS_TERMINATED;
                more = false;
            } else {
                v = v_best - step;
                fp = 0;
                J_prev_same = -1.0;
                if ((rc = extract(dv.best, v))) return fail(rc);
                have_src = true;
            }
        } else {
            // steps 5-6: the augmented level set and the topology at the target
            // the active constraints in the order compliance, stress, eigenvalue, buckling
            const double* grp[4];
            int32_t rows[4];
            double wgt[4], scale[4];
            int nt = 0;
            grp[nt] = dv.S, rows[nt] = nload, wgt[nt] = std::max(mu + gamma * g, 0.0), scale[nt++] = o->alpha_J * J0;
            if (stress)
                grp[nt] = dv.S + (size_t)2 * nload * ne, rows[nt] = nload,
                wgt[nt] = std::max(mu_s + gamma_s * g_s, 0.0), scale[nt++] = o->alpha_sigma * S0;
            if (eigen)
                grp[nt] = dv.SL, rows[nt] = 1, wgt[nt] = std::max(mu_l + gamma_l * g_l, 0.0),
                scale[nt++] = o->alpha_lambda * L0;
            if (buck)
                grp[nt] = dv.SP, rows[nt] = 1, wgt[nt] = std::max(mu_p + gamma_p * g_p, 0.0),
                scale[nt++] = o->alpha_P * P0;
            bool all_zero = true;
            for (int i = 0; i < nt; ++i) all_zero = all_zero && wgt[i] == 0.0;
            double coef[4];
            for (int i = 0; i < nt; ++i) coef[i] = (all_zero ? 1.0 : wgt[i]) / scale[i];
            if ((rc = afd_combine_fields(ctx, ne, nt, grp, rows, coef, dv.raw))) return fail(rc);
            double* cur = dv.raw;
            if (o->damping && have_src) {  // the mean with the level set this topology came from
                const double* g2[2] = {dv.raw, dv.src};
                const int32_t r2[2] = {1, 1};
                const double half[2] = {0.5, 0.5};
                if ((rc = afd_combine_fields(ctx, ne, 2, g2, r2, half, dv.cur))) return fail(rc);
                cur = dv.cur;
            }
            if (event == AFD_LS_CONVERGED) {  // step 8
                v_best = v;
                best_h = solid_h;
                if ((rc = copy(dv.best, cur, ne * sizeof(double), hipMemcpyDeviceToDevice))) return fail(rc);
                if (v - step <= 0.0) {
                    event = AFD_LS_TERMINATED;
                    more = false;
                } else {
                    v -= step;
                    fp = 0;
                    J_prev_same = -1.0;
                    if ((rc = extract(cur, v))) return fail(rc);
                    have_src = true;
                }
            } else {
                J_prev_same = J;
                if ((rc = extract(cur, v))) return fail(rc);
                have_src = true;
            }
        }
        afd_levelset_record& h = hist[k];
        h.fea = k;
        h.event = event;
        h.nsolid = nsolid;
        h.iterations = iters;
        h.v = v_solved;
        h.J = J;
        h.g = g;
        h.mu = mu;
        h.gamma = gamma;
        h.dv = step;
        h.S = Sp;
        h.g_s = g_s;
        h.mu_s = stress ? mu_s : 0.0;
        h.gamma_s = stress ? gamma_s : 0.0;
        h.lam = lam;
        h.g_l = g_l;
        h.mu_l = eigen ? mu_l : 0.0;
        h.gamma_l = eigen ? gamma_l : 0.0;
        h.P = Pb;
        h.g_p = g_p;
        h.mu_p = buck ? mu_p : 0.0;
        h.gamma_p = buck ? gamma_p : 0.0;
        if (hipStreamSynchronize(s) != hipSuccess) {
            set_error("levelset: stream sync failed");
            return fail(AFD_E_HIP);
        }
        h.t_fea = t1 - t0;
        h.t_total = now_s() - t0;
        *n_hist = k + 1;
        if (!more) break;
    }
    memcpy(solid_out, best_h.data(), ne);
    return fail(AFD_OK);
}
