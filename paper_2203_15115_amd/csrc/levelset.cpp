// The augmented topological level-set loop (Sec. 3.2-3.4, 3.6, 3.8; Fig. 6-7):
// Pareto tracing of minimum volume under a hard compliance constraint, as a
// host state machine over the library's device steps (solve, energy fields,
// combined level set, casting projection, ranking).  Every per-element step
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
    double* S = nullptr;        // nload x n_elem energy fields
    double* field = nullptr;    // n_elem, T_L of the last feasible solve
    double* best = nullptr;     // n_elem, T_L of the last converged feasible design
    double* cast = nullptr;     // n_elem, projected field
    int32_t* dist = nullptr;    // n_elem, parting-plane distance
    double* F = nullptr;        // nload x n_dof
    double* U = nullptr;        // nload x n_dof
    double* J = nullptr;        // nload
    void release() {
        for (void* p : {(void*)rho, (void*)solid, (void*)S, (void*)field, (void*)best, (void*)cast, (void*)dist,
                        (void*)F, (void*)U, (void*)J})
            if (p) (void)hipFree(p);
    }
};

template <typename T>
int alloc(T** p, size_t n) {
    if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
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
    Dev dv;
    auto fail = [&](int rc) {
        (void)hipStreamSynchronize(s);
        dv.release();
        return rc;
    };
    int rc = AFD_OK;
    if ((rc = alloc(&dv.rho, ne)) || (rc = alloc(&dv.solid, ne)) || (rc = alloc(&dv.S, (size_t)nload * ne)) ||
        (rc = alloc(&dv.field, ne)) || (rc = alloc(&dv.best, ne)) || (rc = alloc(&dv.cast, ne)) ||
        (rc = alloc(&dv.dist, ne)) || (rc = alloc(&dv.F, (size_t)nload * nd)) ||
        (rc = alloc(&dv.U, (size_t)nload * nd)) || (rc = alloc(&dv.J, nload)))
        return fail(rc);
    if (hipMemcpyAsync(dv.F, F, (size_t)nload * nd * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("levelset: copy of F failed");
        return fail(AFD_E_HIP);
    }
    // topology extraction at volume fraction v from a level-set field
    auto extract = [&](const double* fld, double v) -> int {
        if (o->cast_axis >= 0) {
            AFD_TRY(afd_casting(ctx, dims, fld, o->cast_axis, o->cast_parting, dv.cast, dv.dist));
            return afd_threshold(ctx, dv.cast, dv.dist, ne, v, dv.solid, nullptr, nullptr);
        }
        return afd_threshold(ctx, fld, nullptr, ne, v, dv.solid, nullptr, nullptr);
    };
    // the first topology: the full domain
    std::vector<uint8_t> solid_h(ne, 1), best_h(ne, 1);
    if (hipMemcpyAsync(dv.solid, solid_h.data(), ne, hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("levelset: copy failed");
        return fail(AFD_E_HIP);
    }
    double mu = o->mu0, gamma = o->gamma0, step = o->dv0, v = 1.0, J0 = 0.0, g_prev = 0.0;
    double J_prev_same = -1.0, v_best = 1.0;  // -1: no previous solve at this target
    int fp = 0;
    std::vector<afd_solve_stats> st(nload);
    std::vector<double> Jh(nload);
    const int kmax = std::min(o->max_fea, hist_cap);
    for (int k = 0; k < kmax; ++k) {
        const double t0 = now_s();
        // step 2: the solves over the current topology
        if ((rc = launch_density(ne, dv.solid, o->void_scale, dv.rho, s))) return fail(rc);
        if ((rc = afd_mesh_set_scale(m, dv.rho, ne, AFD_MEM_DEVICE))) return fail(rc);
        afd_solve_opts so = o->solve;
        so.mem_kind = AFD_MEM_DEVICE;
        so.pairs = nullptr;
        so.npairs = 0;
        so.x0 = k > 0 ? dv.U : nullptr;  // warm start from the previous topology's displacements
        if ((rc = afd_solve(m, &so, nload, dv.F, dv.U, dv.J, dv.S, st.data()))) return fail(rc);
        if (hipMemcpyAsync(Jh.data(), dv.J, nload * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(solid_h.data(), dv.solid, ne, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("levelset: copy failed");
            return fail(AFD_E_HIP);
        }
        const double t1 = now_s();
        double J = 0.0;
        int iters = 0;
        for (int r = 0; r < nload; ++r) {
            J += Jh[r];
            iters += st[r].iterations;
        }
        int nsolid = 0;
        for (int64_t e = 0; e < ne; ++e) nsolid += solid_h[e];
        if (topo_hist) memcpy(topo_hist + (size_t)k * ne, solid_h.data(), ne);
        // step 3: constraint value and the multiplier / penalty updates
        if (k == 0) J0 = J;
        const double g = J / (o->alpha_J * J0) - 1.0;
        al_update(mu, gamma, g, g_prev, k, o->varsigma, o->eta);
        g_prev = g;
        ++fp;
        const bool converged = J_prev_same >= 0.0 && std::fabs(J - J_prev_same) < o->conv_tol * J_prev_same;
        int event;
        if (g > 0.0) event = AFD_LS_VIOLATED;                     // step 4
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
            }
        } else {
            // steps 5-6: the augmented level set and the topology at the target
            double w = std::max(mu + gamma * g, 0.0);
            if (w == 0.0) w = 1.0;
            const double coef = w / (o->alpha_J * J0);
            const double* grp[1] = {dv.S};
            const int32_t rows[1] = {nload};
            if ((rc = afd_combine_fields(ctx, ne, 1, grp, rows, &coef, dv.field))) return fail(rc);
            if (event == AFD_LS_CONVERGED) {  // step 8
                v_best = v;
                best_h = solid_h;
                if (hipMemcpyAsync(dv.best, dv.field, ne * sizeof(double), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess) {
                    set_error("levelset: copy failed");
                    return fail(AFD_E_HIP);
                }
                if (v - step <= 0.0) {
                    event = AFD_LS_TERMINATED;
                    more = false;
                } else {
                    v -= step;
                    fp = 0;
                    J_prev_same = -1.0;
                    if ((rc = extract(dv.field, v))) return fail(rc);
                }
            } else {
                J_prev_same = J;
                if ((rc = extract(dv.field, v))) return fail(rc);
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
