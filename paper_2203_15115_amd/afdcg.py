"""Thin ctypes binding of the C ABI in ``include/afdcg.h``.

Argument marshalling only: every step of the solve runs in the HIP library
``libafdcg.so`` (built in-tree by ``build.py``).  Device arrays are passed as
raw pointers (``tensor.data_ptr()`` of torch CUDA tensors); torch is used only
for device memory and streams.  Loading fails loudly when the library is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafdcg.so")

AFD_OK = 0
AFD_PENDING = 1
AFD_E_INVALID_ARG = -1
AFD_E_NO_DEVICE = -2
AFD_E_OOM = -3
AFD_E_OVER_BUDGET = -4
AFD_E_NOT_CONVERGED = -5
AFD_E_BREAKDOWN = -6
AFD_E_COARSE_SINGULAR = -7
AFD_E_HIP = -8
AFD_MEM_HOST = 0
AFD_MEM_DEVICE = 1
AFD_FP64 = 0
AFD_MIXED = 1
AFD_FP32 = 2
AFD_FORM_LAUNCHES = 0
AFD_FORM_PERSISTENT = 1

STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "E_INVALID_ARG", -2: "E_NO_DEVICE", -3: "E_OOM",
                -4: "E_OVER_BUDGET", -5: "E_NOT_CONVERGED", -6: "E_BREAKDOWN",
                -7: "E_COARSE_SINGULAR", -8: "E_HIP"}

EXPORTED = [
    "afd_context_create", "afd_context_destroy", "afd_last_error", "afd_context_sync", "afd_context_use_graphs",
    "afd_mesh_coarse_precision", "afd_mesh_solver_form", "afd_casting",
    "afd_mesh_create", "afd_mesh_destroy", "afd_mesh_sizes", "afd_mesh_set_scale", "afd_mesh_set_fixed",
    "afd_mesh_footprint", "afd_mesh_ke", "afd_apply_K", "afd_apply_K_mfma", "afd_mesh_autotune", "afd_mesh_apply_config",
    "afd_jacobi",
    "afd_dot",
    "afd_restrict", "afd_prolong", "afd_coarse_setup", "afd_coarse_matrix", "afd_coarse_solve",
    "afd_sensitivity", "afd_threshold", "afd_threshold_noalloc", "afd_solve", "afd_combine_fields",
    "afd_levelset_run", "afd_stress_pnorm", "afd_apply_M", "afd_modal", "afd_apply_Kg", "afd_buckling", "afd_server_create", "afd_server_submit",
    "afd_server_poll", "afd_server_wait", "afd_server_clock", "afd_server_destroy",
]


class afd_mesh_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("E", C.c_double), ("nu", C.c_double),
                ("bx", C.c_int32), ("by", C.c_int32), ("bz", C.c_int32)]


class afd_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("inner_rtol", C.c_double), ("check_every", C.c_int32), ("mem_kind", C.c_int32),
                ("pairs", C.POINTER(C.c_int32)), ("npairs", C.c_int32), ("max_refine", C.c_int32),
                ("x0", C.c_void_p)]


class afd_solve_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("refinements", C.c_int32), ("status", C.c_int32),
                ("coarse_dropped", C.c_int32), ("rel_residual_true", C.c_double),
                ("t_setup", C.c_double), ("t_iter", C.c_double), ("t_post", C.c_double)]


class afd_tune_report(C.Structure):
    _fields_ = [("variant", C.c_int32), ("zc", C.c_int32), ("us", C.c_double), ("default_us", C.c_double),
                ("ncandidates", C.c_int32)]


class afd_levelset_opts(C.Structure):
    _fields_ = [("alpha_J", C.c_double), ("dv0", C.c_double), ("dv_min", C.c_double), ("mu0", C.c_double),
                ("gamma0", C.c_double), ("varsigma", C.c_double), ("eta", C.c_double), ("conv_tol", C.c_double),
                ("max_fp", C.c_int32), ("max_fea", C.c_int32), ("void_scale", C.c_double),
                ("cast_axis", C.c_int32), ("cast_parting", C.c_int32), ("alpha_sigma", C.c_double),
                ("pnorm_p", C.c_double), ("damping", C.c_int32), ("solve", afd_solve_opts),
                ("alpha_lambda", C.c_double), ("modal_tol", C.c_double), ("lambda_soft", C.c_int32),
                ("alpha_P", C.c_double), ("P_soft", C.c_int32)]


class afd_levelset_record(C.Structure):
    _fields_ = [("fea", C.c_int32), ("event", C.c_int32), ("nsolid", C.c_int32), ("iterations", C.c_int32),
                ("v", C.c_double), ("J", C.c_double), ("g", C.c_double), ("mu", C.c_double),
                ("gamma", C.c_double), ("dv", C.c_double), ("t_fea", C.c_double), ("t_total", C.c_double),
                ("S", C.c_double), ("g_s", C.c_double), ("mu_s", C.c_double), ("gamma_s", C.c_double),
                ("lam", C.c_double), ("g_l", C.c_double), ("mu_l", C.c_double), ("gamma_l", C.c_double),
                ("P", C.c_double), ("g_p", C.c_double), ("mu_p", C.c_double), ("gamma_p", C.c_double)]


AFD_LS_FIXED_POINT, AFD_LS_CONVERGED, AFD_LS_VIOLATED, AFD_LS_DIVERGED, AFD_LS_TERMINATED = 0, 1, 2, 3, 4


class afd_modal_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("cg_iterations", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double * 3), ("t", C.c_double)]


class afd_request(C.Structure):
    _fields_ = [("desc", afd_mesh_desc), ("rho", C.c_void_p), ("fixed", C.c_void_p), ("F", C.c_void_p),
                ("nrhs", C.c_int32), ("opts", afd_solve_opts)]


class afd_result(C.Structure):
    _fields_ = [("U", C.c_void_p), ("J", C.c_void_p), ("stats", C.c_void_p), ("status", C.c_int32),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run paper_2203_15115_amd/build.py (no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "afd_context_create": (C.c_int, [C.c_int, vp, C.POINTER(vp)]),
            "afd_context_destroy": (None, [vp]),
            "afd_last_error": (C.c_char_p, []),
            "afd_context_sync": (C.c_int, [vp]),
            "afd_context_use_graphs": (C.c_int, [vp, i32]),
            "afd_mesh_coarse_precision": (C.c_int, [vp, i32]),
            "afd_mesh_solver_form": (C.c_int, [vp, i32]),
            "afd_mesh_create": (C.c_int, [vp, C.POINTER(afd_mesh_desc), C.POINTER(vp)]),
            "afd_mesh_destroy": (None, [vp]),
            "afd_mesh_sizes": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
            "afd_mesh_set_scale": (C.c_int, [vp, vp, i64, C.c_int]),
            "afd_mesh_set_fixed": (C.c_int, [vp, vp, i64, C.c_int]),
            "afd_mesh_footprint": (C.c_int, [vp, i32, i32, C.POINTER(C.c_uint64)]),
            "afd_mesh_ke": (C.c_int, [vp, vp]),
            "afd_apply_K": (C.c_int, [vp, i32, i32, vp, vp]),
            "afd_apply_K_mfma": (C.c_int, [vp, i32, vp, vp]),
            "afd_mesh_autotune": (C.c_int, [vp, i32, i32, C.POINTER(afd_tune_report)]),
            "afd_mesh_apply_config": (C.c_int, [vp, i32, i32, i32]),
            "afd_jacobi": (C.c_int, [vp, vp]),
            "afd_dot": (C.c_int, [vp, i64, vp, vp, vp]),
            "afd_restrict": (C.c_int, [vp, i32, vp, vp]),
            "afd_prolong": (C.c_int, [vp, i32, vp, vp]),
            "afd_coarse_setup": (C.c_int, [vp, C.POINTER(i32)]),
            "afd_coarse_matrix": (C.c_int, [vp, vp]),
            "afd_coarse_solve": (C.c_int, [vp, i32, vp, vp]),
            "afd_sensitivity": (C.c_int, [vp, i32, vp, i32, vp, vp]),
            "afd_threshold": (C.c_int, [vp, vp, vp, i64, dbl, vp, vp, C.POINTER(dbl)]),
            "afd_threshold_noalloc": (C.c_int, [vp, vp, vp, i64, dbl, vp, vp, C.POINTER(dbl)]),
            "afd_casting": (C.c_int, [vp, C.POINTER(i32), vp, i32, i32, vp, vp]),
            "afd_solve": (C.c_int, [vp, C.POINTER(afd_solve_opts), i32, vp, vp, vp, vp, vp]),
            "afd_combine_fields": (C.c_int, [vp, i64, i32, vp, vp, vp, vp]),
            "afd_stress_pnorm": (C.c_int, [vp, i32, vp, dbl, vp, C.POINTER(dbl), vp]),
            "afd_apply_M": (C.c_int, [vp, i32, vp, vp]),
            "afd_apply_Kg": (C.c_int, [vp, vp, i32, vp, vp]),
            "afd_buckling": (C.c_int, [vp, vp, C.POINTER(afd_solve_opts), i32, dbl, i32, vp, vp, vp,
                                       C.POINTER(afd_modal_stats)]),
            "afd_modal": (C.c_int, [vp, C.POINTER(afd_solve_opts), i32, dbl, i32, vp, vp, vp,
                                    C.POINTER(afd_modal_stats)]),
            "afd_levelset_run": (C.c_int, [vp, C.POINTER(afd_levelset_opts), i32, vp, vp, vp, i32,
                                           C.POINTER(i32), vp]),
            "afd_server_create": (C.c_int, [vp, C.c_uint64, i32, C.POINTER(vp)]),
            "afd_server_submit": (C.c_int, [vp, C.POINTER(afd_request), C.POINTER(afd_result),
                                            C.POINTER(C.c_uint64)]),
            "afd_server_poll": (C.c_int, [vp, C.c_uint64]),
            "afd_server_wait": (C.c_int, [vp, C.c_uint64, dbl]),
            "afd_server_clock": (dbl, [vp]),
            "afd_server_destroy": (None, [vp]),
        }
        # every exported call is declared: an undeclared one would pass
        # pointers as C ints
        missing = sorted(set(EXPORTED) - set(sig))
        if missing:
            raise RuntimeError(f"no ctypes prototype for {missing}")
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class AfdError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().afd_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, where):
    if code not in (AFD_OK,):
        raise AfdError(code, where)
    return code


def _ptr(x):
    """Raw pointer of a torch tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(type(x))


# ---- same-name wrappers (raise on error) ---------------------------------
def afd_context_create(device=0, stream=None):
    out = C.c_void_p()
    check(lib().afd_context_create(device, stream, C.byref(out)), "afd_context_create")
    return out.value


def afd_context_destroy(ctx):
    lib().afd_context_destroy(ctx)


def afd_context_sync(ctx):
    check(lib().afd_context_sync(ctx), "afd_context_sync")


def afd_context_use_graphs(ctx, enable):
    check(lib().afd_context_use_graphs(ctx, 1 if enable else 0), "afd_context_use_graphs")


def afd_mesh_coarse_precision(mesh, precision):
    check(lib().afd_mesh_coarse_precision(mesh, int(precision)), "afd_mesh_coarse_precision")


def afd_mesh_solver_form(mesh, form):
    check(lib().afd_mesh_solver_form(mesh, int(form)), "afd_mesh_solver_form")


def afd_mesh_create(ctx, dims, h=(1.0, 1.0, 1.0), E=1.0, nu=0.3, block=(0, 0, 0)):
    d = afd_mesh_desc(int(dims[0]), int(dims[1]), int(dims[2]), float(h[0]), float(h[1]), float(h[2]),
                      float(E), float(nu), int(block[0]), int(block[1]), int(block[2]))
    out = C.c_void_p()
    check(lib().afd_mesh_create(ctx, C.byref(d), C.byref(out)), "afd_mesh_create")
    return out.value


def afd_mesh_destroy(mesh):
    lib().afd_mesh_destroy(mesh)


def afd_mesh_sizes(mesh):
    v = [C.c_int64() for _ in range(4)]
    check(lib().afd_mesh_sizes(mesh, *[C.byref(x) for x in v]), "afd_mesh_sizes")
    return tuple(x.value for x in v)


def afd_mesh_set_scale(mesh, rho, n, mem_kind):
    check(lib().afd_mesh_set_scale(mesh, _ptr(rho), n, mem_kind), "afd_mesh_set_scale")


def afd_mesh_set_fixed(mesh, mask, n, mem_kind):
    check(lib().afd_mesh_set_fixed(mesh, _ptr(mask), n, mem_kind), "afd_mesh_set_fixed")


def afd_mesh_footprint(mesh, nrhs, precision):
    b = C.c_uint64()
    check(lib().afd_mesh_footprint(mesh, nrhs, precision, C.byref(b)), "afd_mesh_footprint")
    return b.value


def afd_mesh_ke(mesh, ke_host):
    check(lib().afd_mesh_ke(mesh, _ptr(ke_host)), "afd_mesh_ke")


def afd_apply_K(mesh, precision, nrhs, U, Y):
    check(lib().afd_apply_K(mesh, precision, nrhs, _ptr(U), _ptr(Y)), "afd_apply_K")


def afd_apply_K_mfma(mesh, nrhs, U, Y):
    check(lib().afd_apply_K_mfma(mesh, nrhs, _ptr(U), _ptr(Y)), "afd_apply_K_mfma")


def afd_mesh_autotune(mesh, precision, nrhs):
    """Times the apply candidates on this mesh and keeps the fastest; returns the report."""
    rep = afd_tune_report()
    check(lib().afd_mesh_autotune(mesh, precision, nrhs, C.byref(rep)), "afd_mesh_autotune")
    return rep


def afd_mesh_apply_config(mesh, precision, variant, zc=0):
    check(lib().afd_mesh_apply_config(mesh, precision, variant, zc), "afd_mesh_apply_config")


def afd_jacobi(mesh, d):
    check(lib().afd_jacobi(mesh, _ptr(d)), "afd_jacobi")


def afd_dot(ctx, n, x, y, out):
    check(lib().afd_dot(ctx, n, _ptr(x), _ptr(y), _ptr(out)), "afd_dot")


def afd_restrict(mesh, nrhs, V, G):
    check(lib().afd_restrict(mesh, nrhs, _ptr(V), _ptr(G)), "afd_restrict")


def afd_prolong(mesh, nrhs, MU, V):
    check(lib().afd_prolong(mesh, nrhs, _ptr(MU), _ptr(V)), "afd_prolong")


def afd_coarse_setup(mesh):
    d = C.c_int32()
    check(lib().afd_coarse_setup(mesh, C.byref(d)), "afd_coarse_setup")
    return d.value


def afd_coarse_matrix(mesh, E_host):
    check(lib().afd_coarse_matrix(mesh, _ptr(E_host)), "afd_coarse_matrix")


def afd_coarse_solve(mesh, nrhs, G, MU):
    check(lib().afd_coarse_solve(mesh, nrhs, _ptr(G), _ptr(MU)), "afd_coarse_solve")


def afd_sensitivity(mesh, nrhs, U, pairs, S):
    npairs = len(pairs)
    arr = (C.c_int32 * max(1, 2 * npairs))(*[int(v) for p in pairs for v in p])
    check(lib().afd_sensitivity(mesh, nrhs, _ptr(U), npairs, C.cast(arr, C.c_void_p), _ptr(S)),
          "afd_sensitivity")


def afd_threshold(ctx, s, n, vol_frac, solid, order=None, tie=None):
    tau = C.c_double()
    check(lib().afd_threshold(ctx, _ptr(s), _ptr(tie), n, float(vol_frac), _ptr(solid), _ptr(order),
                              C.byref(tau)), "afd_threshold")
    return tau.value


AFD_THRESHOLD_NOALLOC_MAX = 2097152


def afd_threshold_noalloc(ctx, s, n, vol_frac, solid, order=None, tie=None):
    tau = C.c_double()
    check(lib().afd_threshold_noalloc(ctx, _ptr(s), _ptr(tie), n, float(vol_frac), _ptr(solid), _ptr(order),
                                      C.byref(tau)), "afd_threshold_noalloc")
    return tau.value


def afd_casting(ctx, dims, phi, axis, parting, out, dist=None):
    d = (C.c_int32 * 3)(*[int(x) for x in dims])
    check(lib().afd_casting(ctx, d, _ptr(phi), int(axis), int(parting), _ptr(out), _ptr(dist)), "afd_casting")


def make_opts(rtol=1e-8, max_iter=20000, precision=AFD_FP64, inner_rtol=1e-4, check_every=16,
              mem_kind=AFD_MEM_HOST, pairs=(), max_refine=30, x0=None):
    """x0: start (numpy array or torch tensor per mem_kind, nrhs x n_dof) or None."""
    npairs = len(pairs)
    arr = (C.c_int32 * max(1, 2 * npairs))(*[int(v) for p in pairs for v in p])
    o = afd_solve_opts(float(rtol), int(max_iter), int(precision), float(inner_rtol), int(check_every),
                       int(mem_kind), C.cast(arr, C.POINTER(C.c_int32)), npairs, int(max_refine), _ptr(x0))
    o._keep = (arr, x0)  # keep the pair array and the start alive with the struct
    return o


def afd_solve(mesh, opts, nrhs, F, U, J=None, S=None, raise_on_error=True):
    """Returns (status, [afd_solve_stats] * nrhs)."""
    st = (afd_solve_stats * nrhs)()
    code = lib().afd_solve(mesh, C.byref(opts), nrhs, _ptr(F), _ptr(U), _ptr(J), _ptr(S),
                           C.cast(st, C.c_void_p))
    if raise_on_error:
        check(code, "afd_solve")
    return code, list(st)


def afd_stress_pnorm(mesh, nrhs, U, p=8.0, vm=None, B=None):
    """Returns the p-norm of the von Mises stresses of the nrhs fields."""
    pn = C.c_double()
    check(lib().afd_stress_pnorm(mesh, nrhs, _ptr(U), float(p), _ptr(vm), C.byref(pn), _ptr(B)), "afd_stress_pnorm")
    return pn.value


def afd_apply_M(mesh, nrhs, U, Y):
    check(lib().afd_apply_M(mesh, nrhs, _ptr(U), _ptr(Y)), "afd_apply_M")


def afd_modal(mesh, inner, nev, Phi, S=None, tol=1e-8, max_iter=60, raise_on_error=True):
    """Returns (status, eigenvalues list, afd_modal_stats)."""
    lam = (C.c_double * nev)()
    st = afd_modal_stats()
    code = lib().afd_modal(mesh, C.byref(inner), nev, float(tol), int(max_iter), C.cast(lam, C.c_void_p), _ptr(Phi),
                           _ptr(S), C.byref(st))
    if raise_on_error:
        check(code, "afd_modal")
    return code, list(lam), st


def afd_apply_Kg(mesh, U0, nrhs, X, Y):
    check(lib().afd_apply_Kg(mesh, _ptr(U0), nrhs, _ptr(X), _ptr(Y)), "afd_apply_Kg")


def afd_buckling(mesh, U, inner, nev, Phi, S=None, tol=1e-8, max_iter=60, raise_on_error=True):
    """Returns (status, load factors list, afd_modal_stats)."""
    lam = (C.c_double * nev)()
    st = afd_modal_stats()
    code = lib().afd_buckling(mesh, _ptr(U), C.byref(inner), nev, float(tol), int(max_iter), C.cast(lam, C.c_void_p),
                              _ptr(Phi), _ptr(S), C.byref(st))
    if raise_on_error:
        check(code, "afd_buckling")
    return code, list(lam), st


def afd_combine_fields(ctx, n, groups, coef, out):
    """groups: sequence of (device tensor of rows x n, rows) pairs; coef: one value per group."""
    k = len(groups)
    ptrs = (C.c_void_p * k)(*[_ptr(g) for g, _ in groups])
    rows = (C.c_int32 * k)(*[int(r) for _, r in groups])
    cf = (C.c_double * k)(*[float(c) for c in coef])
    check(lib().afd_combine_fields(ctx, n, k, C.cast(ptrs, C.c_void_p), C.cast(rows, C.c_void_p),
                                   C.cast(cf, C.c_void_p), _ptr(out)), "afd_combine_fields")


def make_levelset_opts(alpha_J=3.0, dv0=0.025, dv_min=0.025 / 16, mu0=100.0, gamma0=10.0, varsigma=0.25, eta=10.0,
                       conv_tol=0.01, max_fp=8, max_fea=400, void_scale=1e-3, cast_axis=-1, cast_parting=0,
                       alpha_sigma=0.0, pnorm_p=8.0, damping=False, alpha_lambda=0.0, modal_tol=1e-9,
                       lambda_soft=False, alpha_P=0.0, P_soft=False, **solvekw):
    so = make_opts(**solvekw)
    o = afd_levelset_opts(float(alpha_J), float(dv0), float(dv_min), float(mu0), float(gamma0), float(varsigma),
                          float(eta), float(conv_tol), int(max_fp), int(max_fea), float(void_scale), int(cast_axis),
                          int(cast_parting), float(alpha_sigma), float(pnorm_p), 1 if damping else 0, so,
                          float(alpha_lambda), float(modal_tol), 1 if lambda_soft else 0, float(alpha_P),
                          1 if P_soft else 0)
    o._keep = so._keep
    return o


def afd_levelset_run(mesh, opts, F, nelem, hist_cap=400, with_topologies=False, raise_on_error=True):
    """Returns (status, solid uint8 array, [afd_levelset_record], topologies or None)."""
    import numpy as np
    F = np.ascontiguousarray(np.atleast_2d(F), dtype=np.float64)
    solid = np.zeros(nelem, dtype=np.uint8)
    hist = (afd_levelset_record * hist_cap)()
    n = C.c_int32()
    topo = np.zeros((hist_cap, nelem), dtype=np.uint8) if with_topologies else None
    code = lib().afd_levelset_run(mesh, C.byref(opts), F.shape[0], _ptr(F), _ptr(solid), C.cast(hist, C.c_void_p),
                                  hist_cap, C.byref(n), _ptr(topo))
    if raise_on_error:
        check(code, "afd_levelset_run")
    recs = list(hist)[: n.value]
    return code, solid, recs, (topo[: n.value] if topo is not None else None)


def afd_server_create(ctx, hbm_budget=0, max_slots=4):
    out = C.c_void_p()
    check(lib().afd_server_create(ctx, int(hbm_budget), int(max_slots), C.byref(out)), "afd_server_create")
    return out.value


class ServerRequest:
    """Holds a request's host buffers and result storage alive until it completes."""

    def __init__(self, dims, rho, fixed, F, block=(8, 8, 8), h=(1.0, 1.0, 1.0), E=1.0, nu=0.3, keep_U=True,
                 **optkw):
        import numpy as np
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
        self.F = np.ascontiguousarray(np.atleast_2d(F), dtype=np.float64)
        self.nrhs = self.F.shape[0]
        self.U = np.zeros_like(self.F) if keep_U else None
        self.J = np.zeros(self.nrhs)
        self.stats = (afd_solve_stats * self.nrhs)()
        self.opts = make_opts(**optkw)
        desc = afd_mesh_desc(int(dims[0]), int(dims[1]), int(dims[2]), float(h[0]), float(h[1]), float(h[2]),
                             float(E), float(nu), int(block[0]), int(block[1]), int(block[2]))
        self.req = afd_request(desc, self.rho.ctypes.data, self.fixed.ctypes.data, self.F.ctypes.data,
                               self.nrhs, self.opts)
        self.res = afd_result(None if self.U is None else self.U.ctypes.data, self.J.ctypes.data,
                              C.cast(self.stats, C.c_void_p).value, AFD_PENDING, 0.0, 0.0, 0.0)
        self.ticket = None


def afd_server_submit(srv, sreq):
    t = C.c_uint64()
    check(lib().afd_server_submit(srv, C.byref(sreq.req), C.byref(sreq.res), C.byref(t)), "afd_server_submit")
    sreq.ticket = t.value
    return t.value


def afd_server_poll(srv, ticket):
    return lib().afd_server_poll(srv, ticket)


def afd_server_wait(srv, ticket, timeout_s=-1.0):
    return lib().afd_server_wait(srv, ticket, float(timeout_s))


def afd_server_clock(srv):
    return lib().afd_server_clock(srv)


def afd_server_destroy(srv):
    lib().afd_server_destroy(srv)
