"""Benchmark of the assembly-free deflated voxel solve on one MI355X.

Workload: the 192x96x96 voxel cantilever (1,769,472 hex8 elements,
5,447,811 DOF), 50% void from a seeded smooth random field thresholded at its
median, clamped on x=0, unit -z load on the x=L bottom edge, 8x8x8 deflation
blocks, FP64, relative residual 1e-8.  Inputs are synthetic (seeded) and
resident in HBM before timing starts.

A step is one pass of the whole hot path from device-resident inputs:
density and fixity made current, Jacobi diagonal, coarse matrix W^T K W and
its factor, deflated PCG to 1e-8, compliance, strain-energy sensitivity field
and topology extraction at a volume fraction.  The headline
value is the throughput of the element-by-element operator apply (GDOF/s =
DOFs / time per apply), timed with HIP events on the stream the library
launches on; the roofline object prices that kernel against HBM.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per FP64 apply launch at 192x96x96 from rocprofv3 FETCH_SIZE + WRITE_SIZE, each scaled by the
# same counter on a 512 MiB copy (kernel as of the committed counter summary
# profiles/apply_fp64_192x96x96_counters.md); None when not measured
TRAFFIC_BYTES = 74_861_517 + 43_919_251


# plain-apply kernel of each autotuner variant
KERNEL_NAMES = {0: "k_matvec<double, APPLY, cubic>", 2: "k_apply_tm<double, cubic, 1>",
                3: "k_apply_tm<double, cubic, 2>", 4: "k_apply_bl<double, cubic, 2>",
                6: "k_apply_bl<double, cubic, 1>", -1: "k_apply_bl<double, cubic, 1>"}


def matvec_algorithmic_bytes(dims, word=8):
    """Bytes the apply must move: read u and write y (3 words per node each),
    one fixity byte per node, one density word per element."""
    nx, ny, nz = dims
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    ne = nx * ny * nz
    return nn * (6 * word + 1) + ne * word


def cpu_baseline(budget_s=12.0):
    """The CPU oracle, as it stands, on the GPU machine's host: its
    element-by-element product K.u (rho_e Ke u_e gathered and scattered with
    numpy, one core) on the full 192x96x96 workload (the value, GDOF/s);
    beside it the oracle's assembled CSR product on the 96x48x48 replica, and
    its direct solve (SuperLU) and deflated CG to 1e-8 on the 24x12x12
    workload.  numpy's einsum and scipy's CSR product and SuperLU run on one
    thread."""
    import scipy
    from oracle import fem, solvers
    from paper_2203_15115_amd import workloads as wl
    Ke = fem.ke_gauss()
    p = wl.config(1)
    u = np.random.default_rng(0).standard_normal(p.ndof)
    reps, t0 = 0, time.perf_counter()
    while True:
        fem.apply_ebe(p.dims, p.rho, Ke, u)
        reps += 1
        if time.perf_counter() - t0 > budget_s and reps >= 2:
            break
    t_ebe = (time.perf_counter() - t0) / reps
    q = wl.cantilever((96, 48, 48), 50, seed=1001, ell=8.0, block=(8, 8, 8))
    t0 = time.perf_counter()
    K = fem.assemble(q.dims, q.rho, Ke)
    t_asm = time.perf_counter() - t0
    uq = np.random.default_rng(0).standard_normal(q.ndof)
    nrep, t0 = 0, time.perf_counter()
    while nrep < 3 or time.perf_counter() - t0 < 3.0:
        K @ uq
        nrep += 1
    t_csr = (time.perf_counter() - t0) / nrep
    c = wl.config(0)
    K0 = fem.assemble(c.dims, c.rho, Ke)
    t0 = time.perf_counter()
    solvers.solve_direct(K0, c.fixed, c.F[0])
    t_direct = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it_dcg, _ = solvers.dcg(K0, c.fixed, c.F[0], c.dims, c.block, rtol=1e-8)
    t_dcg = time.perf_counter() - t0
    return {"value": round(p.ndof / t_ebe / 1e9, 5), "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle element-by-element K.u (numpy, 1 thread) on the full 192x96x96 workload "
                      f"({p.ndof} DOF): {t_ebe:.2f} s per product, mean of {reps}",
            "csr_96x48x48_gdofs": round(q.ndof / t_csr / 1e9, 4),
            "csr_96x48x48_note": f"assembled CSR ({K.nnz} nonzeros, assembly {t_asm:.1f} s), scipy "
                                 f"{scipy.__version__} single-threaded SpMV, mean of {nrep}",
            "direct_24x12x12_s": round(t_direct, 3), "dcg_24x12x12_to_1e-8_s": round(t_dcg, 3),
            "dcg_24x12x12_iterations": int(it_dcg)}


def bench_small_solve(ctx, stream):
    """The 24x12x12 workload (12,675 DOF, 4^3 blocks): FP64 deflated solve
    to 1e-8 (time after a warm-up solve on the same mesh)."""
    import torch
    from paper_2203_15115_amd import afdcg, workloads as wl
    p = wl.config(0)
    m = afdcg.afd_mesh_create(ctx, p.dims, block=p.block)
    afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)
    afdcg.afd_mesh_set_fixed(m, p.fixed, p.ndof, afdcg.AFD_MEM_HOST)
    F = torch.as_tensor(p.F, device="cuda").contiguous()
    U = torch.empty_like(F)
    opts = afdcg.make_opts(rtol=1e-8, mem_kind=afdcg.AFD_MEM_DEVICE)
    afdcg.afd_solve(m, opts, 1, F, U)
    ts = []
    for _ in range(5):
        afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)  # setup included
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = afdcg.afd_solve(m, opts, 1, F, U)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    afdcg.afd_mesh_destroy(m)
    return {"workload": "cantilever 24x12x12, 30% void, 4x4x4 blocks, FP64 to 1e-8",
            "time_to_1e-8_s": round(sorted(ts)[2], 5), "iterations": st[0].iterations,
            "rel_residual_true": st[0].rel_residual_true}


def mixed_vs_oracle(ctx, stream):
    """Mixed-precision solve of the 32x16x16 replica of the 256x128x128
    recipe (50% void, 8^3 blocks, rtol 1e-11) against the oracle's direct
    solve of the assembled system: relative displacement error."""
    import torch
    from oracle import fem, solvers
    from paper_2203_15115_amd import afdcg, workloads as wl
    p = wl.cantilever((32, 16, 16), 50, seed=1003, block=(8, 8, 8))
    m = afdcg.afd_mesh_create(ctx, p.dims, block=p.block)
    afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)
    afdcg.afd_mesh_set_fixed(m, p.fixed, p.ndof, afdcg.AFD_MEM_HOST)
    out = {"workload": "cantilever 32x16x16 (the 256x128x128 recipe at 1/8 per axis), direct oracle"}
    U = np.zeros((1, p.ndof))
    for name, prec, rtol in (("mixed_1e-11", afdcg.AFD_MIXED, 1e-11), ("mixed_1e-8", afdcg.AFD_MIXED, 1e-8),
                             ("fp64_1e-8", afdcg.AFD_FP64, 1e-8)):
        afdcg.afd_solve(m, afdcg.make_opts(rtol=rtol, precision=prec), 1, np.ascontiguousarray(p.F), U)
        out[name] = U[0].copy()
    afdcg.afd_mesh_destroy(m)
    ud = solvers.solve_direct(fem.assemble(p.dims, p.rho, fem.ke_gauss()), p.fixed, p.F[0])
    for k in ("mixed_1e-11", "mixed_1e-8", "fp64_1e-8"):
        out[k] = float(np.linalg.norm(out[k] - ud) / np.linalg.norm(ud))
    return out


def _events_time(stream, fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        fn()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def bench_multi(ctx, stream, args):
    """128x64x64, 40% void level-set field, 4 right-hand sides (bottom, mid and
    top edge loads + one point load standing for an adjoint load): operator
    apply on VALU (Haar-factored) vs on the FP64 matrix cores (dense 24x24
    contraction), and the 4-RHS deflated solve with energies and mutual
    energies."""
    import torch
    from paper_2203_15115_amd import afdcg, workloads as wl
    p = wl.config(2)
    dev = torch.device("cuda:0")
    m = afdcg.afd_mesh_create(ctx, p.dims, block=p.block)
    afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)
    afdcg.afd_mesh_set_fixed(m, p.fixed, p.ndof, afdcg.AFD_MEM_HOST)
    U = torch.randn((4, p.ndof), dtype=torch.float64, device=dev)
    Y = torch.empty_like(U)
    for _ in range(500):  # clocks ramp up over the first few hundred launches
        afdcg.afd_apply_K(m, afdcg.AFD_FP64, 4, U, Y)
    t_valu = _events_time(stream, lambda: afdcg.afd_apply_K(m, afdcg.AFD_FP64, 4, U, Y), 50)
    t_one = _events_time(stream, lambda: afdcg.afd_apply_K(m, afdcg.AFD_FP64, 1, U[0], Y[0]), 50)
    # the autotuner's pick for 4 columns (the solver's plain applies use it)
    rep = afdcg.afd_mesh_autotune(m, afdcg.AFD_FP64, 4)
    t_tuned = _events_time(stream, lambda: afdcg.afd_apply_K(m, afdcg.AFD_FP64, 4, U, Y), 50)
    # algorithmic bytes of the 4-column apply: u and y of every column, densities and fixity once
    nn = (p.dims[0] + 1) * (p.dims[1] + 1) * (p.dims[2] + 1)
    alg4 = matvec_algorithmic_bytes(p.dims) + 3 * nn * 6 * 8
    t_mfma = _events_time(stream, lambda: afdcg.afd_apply_K_mfma(m, 4, U, Y), 50)
    nx, ny, nz = p.dims
    # dense contraction flops actually issued: 32 (padded) x 24 x 2 per element per RHS,
    # over the overlapped tiles (16x16 element tiles owning 15x15 nodes)
    alg_flops = 4 * p.nelem * 24 * 24 * 2
    F = torch.as_tensor(p.F, device=dev).contiguous()
    Uo = torch.empty_like(F)
    J = torch.empty(4, dtype=torch.float64, device=dev)
    pairs = ((0, 3), (1, 3), (2, 3))
    S = torch.empty((7, p.nelem), dtype=torch.float64, device=dev)
    opts = afdcg.make_opts(rtol=1e-8, mem_kind=afdcg.AFD_MEM_DEVICE, pairs=pairs, check_every=32)
    afdcg.afd_coarse_setup(m)
    afdcg.afd_solve(m, opts, 4, F, Uo, J, S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = afdcg.afd_solve(m, opts, 4, F, Uo, J, S)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    Jh = J.cpu().numpy()
    Fh = p.F
    Uh = Uo.cpu().numpy()
    recip = max(abs(Fh[a] @ Uh[b] - Fh[b] @ Uh[a]) / abs(Fh[a] @ Uh[b]) for a, b in pairs)
    afdcg.afd_mesh_destroy(m)
    return {"workload": "cantilever 128x64x64, 40% void, 4 RHS (3 edge loads + point load), 8x8x8 blocks",
            "apply_valu_us": round(t_valu * 1e6, 2), "apply_mfma_us": round(t_mfma * 1e6, 2),
            "apply_valu_1rhs_us": round(t_one * 1e6, 2), "apply_4rhs_over_4x1rhs": round(t_valu / (4 * t_one), 3),
            "apply_valu_tuned_us": round(t_tuned * 1e6, 2), "tuned_config": {"variant": rep.variant, "zc": rep.zc},
            "apply_4rhs_tuned_hbm_frac": round(alg4 / t_tuned / 1e9 / HBM_PEAK_GBS, 4),
            "apply_4rhs_alg_bytes": alg4, "apply_4rhs_hbm_frac": round(alg4 / t_valu / 1e9 / HBM_PEAK_GBS, 4),
            "gdofs_valu_total": round(4 * p.ndof / t_valu / 1e9, 2),
            "gdofs_mfma_total": round(4 * p.ndof / t_mfma / 1e9, 2),
            "mfma_tflops": round(alg_flops / t_mfma / 1e12, 3), "mfma_peak_tflops": 78.6,
            "mfma_frac": round(alg_flops / t_mfma / 1e12 / 78.6, 4),
            "solve_4rhs_s": round(t_solve, 4), "iterations": [x.iterations for x in st],
            "rel_residual_true": [x.rel_residual_true for x in st],
            "compliance": [float(v) for v in Jh], "reciprocity_rel_err": float(recip)}


def bench_mixed(ctx, stream, args):
    """256x128x128 (12.8M DOF), 50% void: FP32-inner / FP64-refined deflated
    solve to 1e-8 against the FP64 deflated solve of the same system."""
    import torch
    from paper_2203_15115_amd import afdcg, workloads as wl
    p = wl.config(3)
    dev = torch.device("cuda:0")
    m = afdcg.afd_mesh_create(ctx, p.dims, block=p.block)
    afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)
    afdcg.afd_mesh_set_fixed(m, p.fixed, p.ndof, afdcg.AFD_MEM_HOST)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    afdcg.afd_coarse_setup(m)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    F = torch.as_tensor(p.F, device=dev).contiguous()
    out = {"workload": "cantilever 256x128x128, 50% void, 8x8x8 blocks, rtol 1e-8", "n_dof": p.ndof,
           "setup_s": round(t_setup, 4)}
    U = {}
    for name, prec in (("fp64", afdcg.AFD_FP64), ("mixed", afdcg.AFD_MIXED)):
        Uo = torch.empty_like(F)
        opts = afdcg.make_opts(rtol=1e-8, precision=prec, mem_kind=afdcg.AFD_MEM_DEVICE, check_every=32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, st = afdcg.afd_solve(m, opts, 1, F, Uo, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        U[name] = Uo
        out[name] = {"time_s": round(dt, 4), "status": code, "iterations": st[0].iterations,
                     "refinements": st[0].refinements, "rel_residual_true": st[0].rel_residual_true}
    d = (U["mixed"] - U["fp64"]).norm().item() / U["fp64"].norm().item()
    out["mixed_vs_fp64_rel_diff"] = d
    out["speedup_mixed_over_fp64"] = round(out["fp64"]["time_s"] / out["mixed"]["time_s"], 3)
    afdcg.afd_mesh_destroy(m)
    return out


def bench_serve(ctx, args):
    """Stream of cantilever requests nx x nx/2 x nx/2, nx uniform in
    {32,...,160}, 20-60% void, 1-4 RHS, to 1e-8: the continuous-batching
    server (mixed precision, 4 slots) against one-at-a-time FP64 solves in
    arrival order (1 slot) on the same GPU.  Each server's saturated
    throughput is measured on the first --serve-sat requests kept queued
    (a bounded backlog of slots + 4); then the same Poisson stream of
    --serve-requests requests, at 0.8x the batched server's saturated rate,
    is served by each, with latencies from submission to completion.
    Request inputs are prepared by a producer thread ahead of their arrival
    (workloads.RequestFactory), and displacements are not copied back (the
    server keeps compliances, residuals and statuses)."""
    import queue
    import threading

    import numpy as np
    from paper_2203_15115_amd import afdcg, workloads as wl
    n = args.serve_requests
    reqs = wl.request_stream(n, rate=0.0, seed=7)
    fac = wl.RequestFactory(seed=7)

    def run_server(prec, slots, count, arrivals=None):
        q = queue.Queue(maxsize=32)

        def produce():
            for r in reqs[:count]:
                p = fac.problem(r)
                q.put(afdcg.ServerRequest(p.dims, p.rho, p.fixed, p.F, block=p.block, rtol=1e-8, precision=prec,
                                          keep_U=False))
        th = threading.Thread(target=produce, daemon=True)
        th.start()
        srv = afdcg.afd_server_create(ctx, 0, slots)
        live, lat, lag, codes, resid = [], [], [], [], []

        def reap(block_until=None):
            keep = []
            for r in live:
                c = afdcg.afd_server_poll(srv, r.ticket)
                if c == afdcg.AFD_PENDING:
                    keep.append(r)
                    continue
                codes.append(c)
                lat.append(r.res.t_done - r.res.t_submit)
                resid.append(max(s.rel_residual_true for s in r.stats))
            live[:] = keep
        t0 = time.perf_counter()
        for i in range(count):
            r = q.get()
            if arrivals is None:  # saturated: keep a bounded backlog queued
                while len(live) >= slots + 4:
                    time.sleep(0.0005)
                    reap()
            else:
                while time.perf_counter() - t0 < arrivals[i]:
                    time.sleep(0.0003)
                    if i % 8 == 0:
                        reap()
                lag.append(time.perf_counter() - t0 - arrivals[i])
            afdcg.afd_server_submit(srv, r)
            live.append(r)
            reap()
        while live:
            time.sleep(0.001)
            reap()
        t_end = time.perf_counter() - t0
        afdcg.afd_server_destroy(srv)
        lat = np.array(lat)
        return {"requests": count, "solves_per_s": round(count / t_end, 3), "elapsed_s": round(t_end, 2),
                "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                "ok": int(sum(c == 0 for c in codes)), "max_rel_residual": float(max(resid)),
                "max_submit_lag_s": round(float(max(lag)), 4) if lag else 0.0}

    out = {"workload": f"{n} Poisson-arrival requests, nx in 32..160, 20-60% void, 1-4 RHS, rtol 1e-8 "
                       f"(saturation on the first {args.serve_sat})"}
    modes = (("batched_mixed_4slots", afdcg.AFD_MIXED, 4), ("fifo_fp64_1slot", afdcg.AFD_FP64, 1))
    for name, prec, slots in modes:
        out[name] = {"saturated": run_server(prec, slots, min(args.serve_sat, n))}
        print(f"# serving: {name} saturated {json.dumps(out[name]['saturated'])}", file=sys.stderr, flush=True)
    rate = 0.8 * out["batched_mixed_4slots"]["saturated"]["solves_per_s"]
    arrivals = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, n))
    out["arrival_rate_per_s"] = round(rate, 3)
    for name, prec, slots in modes:
        out[name]["poisson"] = run_server(prec, slots, n, arrivals)
        print(f"# serving: {name} poisson {json.dumps(out[name]['poisson'])}", file=sys.stderr, flush=True)
    return out


def bench_modal(ctx, stream):
    """The lowest eigenpair of the 128x64x64 cantilever (40% void, 8^3
    blocks) by subspace iteration on 4 vectors with 4-column deflated inner
    solves to 1e-10, with its eigenvalue sensitivity field (Eq. 3.4)."""
    import torch
    from paper_2203_15115_amd import afdcg, workloads as wl
    p = wl.config(2)
    m = afdcg.afd_mesh_create(ctx, p.dims, block=p.block)
    afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)
    afdcg.afd_mesh_set_fixed(m, p.fixed, p.ndof, afdcg.AFD_MEM_HOST)
    afdcg.afd_coarse_setup(m)
    Phi = torch.empty((1, p.ndof), dtype=torch.float64, device="cuda")
    S = torch.empty((1, p.nelem), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    code, lam, st = afdcg.afd_modal(m, afdcg.make_opts(rtol=1e-10, check_every=32), 1, Phi, S, tol=1e-8,
                                    max_iter=60, raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    afdcg.afd_mesh_destroy(m)
    return {"workload": "lowest eigenpair, cantilever 128x64x64, 40% void, 8x8x8 blocks, block of 4, inner "
                        "solves to 1e-10, Ritz residual 1e-8", "status": code, "lambda": lam[0],
            "time_s": round(dt, 4), "subspace_iterations": st.iterations, "cg_iterations": st.cg_iterations,
            "rel_residual": st.rel_residual[0]}


def bench_buckling(ctx, stream):
    """The smallest buckling load factor of the 128x64x64 cantilever (40%
    void, 8^3 blocks) under an axial compression of its free end plus its
    bottom-edge load (Eq. 3.5): the static solve to 1e-10, then subspace
    iteration on 4 vectors with 4-column deflated inner solves to 1e-10 and
    the load-factor sensitivity field."""
    import torch
    from paper_2203_15115_amd import afdcg, workloads as wl
    p = wl.config(2)
    d = p.dims
    f = wl.edge_load(d, "bottom")
    for j in range(d[1] + 1):
        for k in range(d[2] + 1):
            f[3 * wl.node_id(d, d[0], j, k)] -= 1.0 / ((d[1] + 1) * (d[2] + 1))
    m = afdcg.afd_mesh_create(ctx, d, block=p.block)
    afdcg.afd_mesh_set_scale(m, p.rho, p.nelem, afdcg.AFD_MEM_HOST)
    afdcg.afd_mesh_set_fixed(m, p.fixed, p.ndof, afdcg.AFD_MEM_HOST)
    afdcg.afd_coarse_setup(m)
    U = torch.empty((1, p.ndof), dtype=torch.float64, device="cuda")
    Phi = torch.empty((1, p.ndof), dtype=torch.float64, device="cuda")
    S = torch.empty((1, p.nelem), dtype=torch.float64, device="cuda")
    Fd = torch.as_tensor(f[None], device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    afdcg.afd_solve(m, afdcg.make_opts(rtol=1e-10, check_every=32, mem_kind=afdcg.AFD_MEM_DEVICE), 1, Fd, U)
    code, lam, st = afdcg.afd_buckling(m, U, afdcg.make_opts(rtol=1e-10, check_every=32), 1, Phi, S, tol=1e-8,
                                       max_iter=60, raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    afdcg.afd_mesh_destroy(m)
    return {"workload": "smallest buckling load factor, cantilever 128x64x64, 40% void, 8x8x8 blocks, axial "
                        "compression + bottom-edge load, block of 4, inner solves to 1e-10, Ritz residual 1e-8",
            "status": code, "load_factor": lam[0], "time_s": round(dt, 4), "subspace_iterations": st.iterations,
            "cg_iterations": st.cg_iterations, "rel_residual": st.rel_residual[0]}


def bench_levelset(ctx, stream):
    """The augmented topological level-set loop (Sec. 3.8, Fig. 7) on a
    96x48x48 cantilever (221,184 elements, 680,775 DOF, 8^3 blocks) from the
    full domain, bottom-edge load, J <= 3 J0, dv0 = 0.025, solves to 1e-8
    (FP64, warm-started): solves, final volume, time, and the share of the
    time spent in the solves (the paper reports 88% in its Fig. 10)."""
    from paper_2203_15115_amd import afdcg, workloads as wl
    dims = (96, 48, 48)
    n = wl.n_elems(dims)
    m = afdcg.afd_mesh_create(ctx, dims, block=(8, 8, 8))
    afdcg.afd_mesh_set_fixed(m, wl.clamp_x0(dims), 3 * wl.n_nodes(dims), afdcg.AFD_MEM_HOST)
    o = afdcg.make_levelset_opts(alpha_J=3.0, rtol=1e-8, check_every=16)
    t0 = time.perf_counter()
    code, solid, hist, _ = afdcg.afd_levelset_run(m, o, wl.edge_load(dims, "bottom")[None], n, hist_cap=400)
    dt = time.perf_counter() - t0
    afdcg.afd_mesh_destroy(m)
    conv = [r for r in hist if r.event == afdcg.AFD_LS_CONVERGED]
    t_fea = sum(r.t_fea for r in hist)
    out = {"workload": "level-set loop, cantilever 96x48x48, 8x8x8 blocks, J <= 3 J0, FP64 solves to 1e-8",
           "status": code, "solves": len(hist), "volume_steps": len(conv), "final_volume": round(conv[-1].v, 5),
           "final_J_over_J0": round(conv[-1].J / hist[0].J, 4), "time_s": round(dt, 3),
           "ms_per_solve_step": round(1e3 * dt / len(hist), 3), "solve_share": round(t_fea / dt, 4),
           "cg_iterations_mean": round(sum(r.iterations for r in hist) / len(hist), 1),
           "cg_iterations_first": hist[0].iterations}
    # with the p-norm stress constraint (two edge loads, their adjoint solves, damping)
    m = afdcg.afd_mesh_create(ctx, dims, block=(8, 8, 8))
    afdcg.afd_mesh_set_fixed(m, wl.clamp_x0(dims), 3 * wl.n_nodes(dims), afdcg.AFD_MEM_HOST)
    o = afdcg.make_levelset_opts(alpha_J=100.0, alpha_sigma=2.5, dv_min=0.025 / 4, damping=True, rtol=1e-8,
                                 check_every=16)
    F = np.stack([wl.edge_load(dims, "bottom"), wl.edge_load(dims, "mid")])
    t0 = time.perf_counter()
    code, solid, hist, _ = afdcg.afd_levelset_run(m, o, F, n, hist_cap=400)
    dt = time.perf_counter() - t0
    afdcg.afd_mesh_destroy(m)
    conv = [r for r in hist if r.event == afdcg.AFD_LS_CONVERGED]
    out["stress"] = {"workload": "the same mesh, bottom and mid edge loads, J <= 100 J0, sigma_PN(p=8) <= 2.5 "
                                 "sigma_PN0, damping; 2 primal + 2 adjoint solves per step",
                     "status": code, "solves": len(hist), "final_volume": round(conv[-1].v, 5),
                     "final_S_over_S0": round(conv[-1].S / hist[0].S, 4),
                     "final_J_over_J0": round(conv[-1].J / hist[0].J, 4), "time_s": round(dt, 3),
                     "ms_per_step": round(1e3 * dt / len(hist), 3),
                     "solve_share": round(sum(r.t_fea for r in hist) / dt, 4)}
    # with the eigenvalue constraint lambda_1 >= lambda_10 (Eq. 3.21; the lowest
    # eigenpair of every topology by subspace iteration), on a cross-section of
    # unequal sides so that lambda_1 stays simple, loaded at mid-span
    de = (96, 48, 32)
    ne = wl.n_elems(de)
    fe = np.zeros(3 * wl.n_nodes(de))
    for j in range(de[1] + 1):
        fe[3 * wl.node_id(de, de[0] // 2, j, 0) + 2] = -1.0 / (de[1] + 1)
    m = afdcg.afd_mesh_create(ctx, de, block=(8, 8, 8))
    afdcg.afd_mesh_set_fixed(m, wl.clamp_x0(de), 3 * wl.n_nodes(de), afdcg.AFD_MEM_HOST)
    o = afdcg.make_levelset_opts(alpha_J=3.0, alpha_lambda=1.0, damping=True, dv_min=0.025 / 4, modal_tol=1e-6,
                                 rtol=1e-8, check_every=16)
    t0 = time.perf_counter()
    code, solid, hist, _ = afdcg.afd_levelset_run(m, o, fe[None], ne, hist_cap=400, raise_on_error=False)
    dt = time.perf_counter() - t0
    afdcg.afd_mesh_destroy(m)
    conv = [r for r in hist if r.event == afdcg.AFD_LS_CONVERGED]
    out["eigen"] = {"workload": "cantilever 96x48x32, 8x8x8 blocks, mid-span load, J <= 3 J0, lambda_1 >= lambda_10, "
                                "damping; one FP64 solve to 1e-8 and the lowest eigenpair (Ritz residual 1e-6) per step",
                    "status": code, "solves": len(hist), "final_volume": round(conv[-1].v, 5) if conv else None,
                    "final_lambda_over_lambda0": round(conv[-1].lam / hist[0].lam, 4) if conv else None,
                    "final_J_over_J0": round(conv[-1].J / hist[0].J, 4) if conv else None,
                    "eigen_violations": sum(1 for r in hist if r.event == afdcg.AFD_LS_VIOLATED and r.g_l > 0),
                    "time_s": round(dt, 3), "ms_per_step": round(1e3 * dt / max(1, len(hist)), 3),
                    "solve_and_eigen_share": round(sum(r.t_fea for r in hist) / dt, 4)}
    # with the buckling constraint P >= 0.8 P_0 (Eq. 3.21): the same mesh under an
    # axial compression of the free end plus a mid-edge load
    fb = wl.edge_load(de, "mid")
    for j in range(de[1] + 1):
        for k in range(de[2] + 1):
            fb[3 * wl.node_id(de, de[0], j, k)] -= 1.0 / ((de[1] + 1) * (de[2] + 1))
    m = afdcg.afd_mesh_create(ctx, de, block=(8, 8, 8))
    afdcg.afd_mesh_set_fixed(m, wl.clamp_x0(de), 3 * wl.n_nodes(de), afdcg.AFD_MEM_HOST)
    o = afdcg.make_levelset_opts(alpha_J=3.0, alpha_P=0.8, damping=True, dv_min=0.025 / 4, modal_tol=1e-6,
                                 rtol=1e-8, check_every=16)
    t0 = time.perf_counter()
    code, solid, hist, _ = afdcg.afd_levelset_run(m, o, fb[None], ne, hist_cap=400, raise_on_error=False)
    dt = time.perf_counter() - t0
    afdcg.afd_mesh_destroy(m)
    conv = [r for r in hist if r.event == afdcg.AFD_LS_CONVERGED]
    out["buckling"] = {"workload": "cantilever 96x48x32, 8x8x8 blocks, axial compression + mid-edge load, J <= 3 J0, "
                                   "P >= 0.8 P_0, damping; one FP64 solve to 1e-8 and the smallest buckling load "
                                   "factor (Ritz residual 1e-6) per step",
                       "status": code, "solves": len(hist), "final_volume": round(conv[-1].v, 5) if conv else None,
                       "final_P_over_P0": round(conv[-1].P / hist[0].P, 4) if conv else None,
                       "final_J_over_J0": round(conv[-1].J / hist[0].J, 4) if conv else None,
                       "buckling_violations": sum(1 for r in hist if r.event == afdcg.AFD_LS_VIOLATED and r.g_p > 0),
                       "time_s": round(dt, 3), "ms_per_step": round(1e3 * dt / max(1, len(hist)), 3),
                       "solve_and_eigen_share": round(sum(r.t_fea for r in hist) / dt, 4)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=200, help="timed operator applies")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--sections", default="multi,mixed,modal,buckling,levelset,small,serve",
                    help="extra measured sections: multi (4-RHS, VALU vs matrix cores), mixed, modal, buckling, levelset, "
                         "small (24x12x12 solve), serve")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-sat", type=int, default=200, help="requests of each saturated serving run")
    ap.add_argument("--apply-only", action="store_true",
                    help="only a known-size copy and the timed applies (hardware-counter runs)")
    ap.add_argument("--apply-config", default="-1:0",
                    help="with --apply-only: variant:zc of the applies (-1:0 the default; no autotuning)")
    ap.add_argument("--evict", action="store_true",
                    help="with --apply-only: a 512 MiB read before each apply, on three (u, y) pairs in turn")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only; sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2203_15115_amd import afdcg, workloads as wl

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)  # default priority; the library launches on it
    torch.cuda.set_stream(stream)
    p = wl.config(args.config)
    ctx = afdcg.afd_context_create(0, stream.cuda_stream)
    mesh = afdcg.afd_mesh_create(ctx, p.dims, block=p.block)
    rho_d = torch.as_tensor(p.rho, device=dev)
    fix_d = torch.as_tensor(p.fixed, device=dev)
    F_d = torch.as_tensor(p.F[:1], device=dev).contiguous()
    afdcg.afd_mesh_set_scale(mesh, rho_d, p.nelem, afdcg.AFD_MEM_DEVICE)
    afdcg.afd_mesh_set_fixed(mesh, fix_d, p.ndof, afdcg.AFD_MEM_DEVICE)
    torch.cuda.synchronize()
    if args.apply_only:
        # counter runs time one fixed configuration (the autotuner's pick would
        # vary from run to run under counter collection)
        v, zc = (int(x) for x in args.apply_config.split(":"))
        afdcg.afd_mesh_apply_config(mesh, afdcg.AFD_FP64, v, zc)
        a = torch.empty(64 << 20, dtype=torch.float64, device=dev)  # 512 MiB calibration copy
        b = torch.empty_like(a)
        b.copy_(a)
        pairs = [(torch.randn(p.ndof, dtype=torch.float64, device=dev),
                  torch.empty(p.ndof, dtype=torch.float64, device=dev)) for _ in range(3 if args.evict else 1)]
        for i in range(2000 + args.reps):  # 2000 warm-up launches (steady clocks), then the counted ones
            if args.evict:
                b.sum()
            u, y = pairs[i % len(pairs)]
            afdcg.afd_apply_K(mesh, afdcg.AFD_FP64, 1, u, y)
        torch.cuda.synchronize()
        print(json.dumps({"apply_only": True, "copy_bytes": 2 * a.numel() * 8, "reps": args.reps, "warmup": 2000,
                          "evict": args.evict, "apply_config": {"variant": v, "zc": zc}}), flush=True)
        return

    # ---- apply execution picked by the autotuner on this mesh (outside the timed region)
    tune = {}
    for name, prec in (("fp64", afdcg.AFD_FP64), ("fp32", afdcg.AFD_FP32)):
        r = afdcg.afd_mesh_autotune(mesh, prec, 1)
        tune[name] = {"variant": r.variant, "zc": r.zc, "us": round(r.us, 2), "default_us": round(r.default_us, 2),
                      "candidates": r.ncandidates}
    print(f"# autotune: {json.dumps(tune)}", file=sys.stderr, flush=True)

    # ---- operator apply throughput (HIP events on the library's stream).  The
    # launches are recorded as a HIP graph of 20 applies and replayed, so the
    # host's per-call cost (Python, ctypes) does not leave the GPU idle between
    # kernels of ~30 us; one replay is checked against the eager result; after
    # a warm-up of 10,000 applies the median of three timed batches of --reps
    # applies is reported.
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_applies(prec, uu, yy):
        for _ in range(10):
            afdcg.afd_apply_K(mesh, prec, 1, uu, yy)
        stream.synchronize()
        ref = yy.clone()
        per = 20
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                for _ in range(per):
                    afdcg.afd_apply_K(mesh, prec, 1, uu, yy)
            yy.zero_()
            g.replay()
            stream.synchronize()
            assert torch.equal(yy, ref), "graph replay differs from the eager apply"
            # the apply speeds up over the first few hundred launches of a
            # process (35 -> 30 us measured): warm up for ~0.3 s of applies
            for _ in range(500):
                g.replay()
            stream.synchronize()
            nrep = max(1, args.reps // per)
            batches = []
            for _ in range(3):  # three timed batches; the median is reported
                ev0.record(stream)
                for _ in range(nrep):
                    g.replay()
                ev1.record(stream)
                ev1.synchronize()
                batches.append(ev0.elapsed_time(ev1) / 1e3 / (nrep * per))
            print(f"# apply batches (us): {[round(b * 1e6, 2) for b in batches]}", file=sys.stderr, flush=True)
            return sorted(batches)[1], "graph"
        except RuntimeError as e:  # capture unavailable: eager launches
            print(f"# apply timing without a graph: {e}", file=sys.stderr, flush=True)
            ev0.record(stream)
            for _ in range(args.reps):
                afdcg.afd_apply_K(mesh, prec, 1, uu, yy)
            ev1.record(stream)
            ev1.synchronize()
            return ev0.elapsed_time(ev1) / 1e3 / args.reps, "eager"

    def time_evicted(prec, dtype, reps=60):
        # each launch timed alone (HIP events around it on the library's
        # stream), on one of three distinct (u, y) pairs in turn, after a read
        # of 512 MiB that evicts the previous launch's data from the 256 MB
        # MALL and the L2s: the apply reads u, the densities and the fixity from
        # HBM.  (A read leaves clean lines behind; 512 MiB of writes instead
        # leave dirty lines whose write-back would be charged to the apply.)
        pairs = [(torch.randn(p.ndof, device=dev).to(dtype), torch.empty(p.ndof, dtype=dtype, device=dev))
                 for _ in range(3)]
        flush = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for i in range(reps + 10):
            flush.sum()
            uu, yy = pairs[i % 3]
            if i >= 10:
                evs[i - 10][0].record(stream)
            afdcg.afd_apply_K(mesh, prec, 1, uu, yy)
            if i >= 10:
                evs[i - 10][1].record(stream)
        stream.synchronize()
        ts = sorted(a.elapsed_time(b) / 1e3 for a, b in evs)
        return ts[len(ts) // 2], ts[len(ts) // 10], ts[(9 * len(ts)) // 10]

    u = torch.randn(p.ndof, dtype=torch.float64, device=dev)
    y = torch.empty_like(u)
    t_apply, apply_launch = time_applies(afdcg.AFD_FP64, u, y)
    gdofs = p.ndof / t_apply / 1e9
    alg = matvec_algorithmic_bytes(p.dims)
    achieved = alg / t_apply / 1e9
    print(f"# apply: {t_apply * 1e6:.1f} us/launch, {gdofs:.1f} GDOF/s, {achieved:.0f} GB/s algorithmic",
          file=sys.stderr, flush=True)
    t_ev, t_ev10, t_ev90 = time_evicted(afdcg.AFD_FP64, torch.float64)
    achieved_ev = alg / t_ev / 1e9
    print(f"# apply, MALL evicted: {t_ev * 1e6:.1f} us/launch (p10 {t_ev10 * 1e6:.1f}, p90 {t_ev90 * 1e6:.1f}), "
          f"{achieved_ev:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    # FP32 apply (inner operator of the mixed form)
    uf, yf = u.float(), torch.empty(p.ndof, dtype=torch.float32, device=dev)
    t_apply32, _ = time_applies(afdcg.AFD_FP32, uf, yf)

    # ---- full hot-path steps
    U = torch.empty_like(F_d)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    S = torch.empty((1, p.nelem), dtype=torch.float64, device=dev)
    solid = torch.empty(p.nelem, dtype=torch.uint8, device=dev)
    opts = afdcg.make_opts(rtol=1e-8, max_iter=20000, mem_kind=afdcg.AFD_MEM_DEVICE, check_every=32)
    vf = float((p.rho == 1.0).mean()) - 0.025

    def step():
        # the whole hot path from device-resident inputs: density and fixity
        # made current (this invalidates the Jacobi diagonal and the coarse
        # factor), Jacobi + coarse E = W^T K W + block Cholesky, deflated PCG
        # to 1e-8, compliance, sensitivity, topology
        afdcg.afd_mesh_set_scale(mesh, rho_d, p.nelem, afdcg.AFD_MEM_DEVICE)
        afdcg.afd_mesh_set_fixed(mesh, fix_d, p.ndof, afdcg.AFD_MEM_DEVICE)
        code, st = afdcg.afd_solve(mesh, opts, 1, F_d, U, J, S)
        afdcg.afd_threshold(ctx, S, p.nelem, vf, solid)
        return st[0]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(1, args.steps)
    st = stats[-1]
    print(f"# step: {dt * 1e3:.1f} ms (setup {st.t_setup * 1e3:.1f}, iterations {st.t_iter * 1e3:.1f}, "
          f"post {st.t_post * 1e3:.1f}), {st.iterations} iterations, true rel residual "
          f"{st.rel_residual_true:.2e}", file=sys.stderr, flush=True)

    out = {
        "metric": "matrix-free K.u GDOF/s",
        "value": round(gdofs, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded voxel cantilever)",
        "config": {"workload": f"cantilever {p.dims[0]}x{p.dims[1]}x{p.dims[2]} hex8, 50% void, "
                               f"8x8x8 deflation blocks, FP64 deflated PCG to 1e-8",
                   "n_dof": p.ndof, "n_elem": p.nelem},
        "time_to_1e-8_s": round(st.t_setup + st.t_iter, 5),
        "iterations": st.iterations,
        "rel_residual_true": st.rel_residual_true,
        "setup_s": round(st.t_setup, 4),
        "iterations_s": round(st.t_iter, 4),
        "post_s": round(st.t_post, 4),
        "apply_us": round(t_apply * 1e6, 3),
        "apply_launch": apply_launch,
        "apply_fp32_us": round(t_apply32 * 1e6, 3),
        "apply_fp32_gdofs": round(p.ndof / t_apply32 / 1e9, 3),
        "apply_tuning": tune,
        "apply_mall_evicted_us": {"median": round(t_ev * 1e6, 3), "p10": round(t_ev10 * 1e6, 3),
                                  "p90": round(t_ev90 * 1e6, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # each launch alone after a 512 MiB read (inputs read from HBM, not the MALL)
                     "achieved_mall_evicted": round(achieved_ev, 1),
                     "frac_mall_evicted": round(achieved_ev / HBM_PEAK_GBS, 4),
                     # counters were taken on the default configuration (buffer-load kernel,
                     # prefetch distance 1, one-round z chunking)
                     "traffic": TRAFFIC_BYTES if args.config == 1 and tune["fp64"]["variant"] == -1 else None,
                     "kernel": KERNEL_NAMES[tune["fp64"]["variant"]], "bytes_per_launch": alg},
    }
    # casting projection (Sec. 3.7) of the energy field of the last step: one
    # launch reads and writes one FP64 value per element
    cs = torch.empty_like(S)
    cast = {}
    for axis, parting in ((2, 0), (0, p.dims[0] // 2)):
        for _ in range(20):
            afdcg.afd_casting(ctx, p.dims, S, axis, parting, cs)
        ev0.record(stream)
        for _ in range(200):
            afdcg.afd_casting(ctx, p.dims, S, axis, parting, cs)
        ev1.record(stream)
        ev1.synchronize()
        t_c = ev0.elapsed_time(ev1) * 1e-3 / 200
        cast[f"axis{axis}"] = {"parting": parting, "us": round(t_c * 1e6, 2),
                               "gbs": round(2 * 8 * p.nelem / t_c / 1e9, 1)}
    out["casting"] = cast
    # the FP64 iterations' opt-in coarse solve over FP32 copies of the FP64 factor's solve
    # matrices (FP64 vectors and accumulation), same steps
    afdcg.afd_mesh_coarse_precision(mesh, afdcg.AFD_FP32)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st32 = [step() for _ in range(args.steps)][-1]
    torch.cuda.synchronize()
    out["coarse_fp32_copies"] = {"ms_per_step": round((time.perf_counter() - t0) / max(1, args.steps) * 1e3, 3),
                                 "time_to_1e-8_s": round(st32.t_setup + st32.t_iter, 5),
                                 "iterations": st32.iterations, "rel_residual_true": st32.rel_residual_true}
    secs = [x for x in args.sections.split(",") if x]
    afdcg.afd_mesh_destroy(mesh)
    mesh = None
    if "multi" in secs:
        out["multi_rhs"] = bench_multi(ctx, stream, args)
        print(f"# multi-RHS: {json.dumps(out['multi_rhs'])}", file=sys.stderr, flush=True)
    if "mixed" in secs:
        out["mixed"] = bench_mixed(ctx, stream, args)
        print(f"# mixed: {json.dumps(out['mixed'])}", file=sys.stderr, flush=True)
    if "modal" in secs:
        out["modal"] = bench_modal(ctx, stream)
        print(f"# modal: {json.dumps(out['modal'])}", file=sys.stderr, flush=True)
    if "buckling" in secs:
        out["buckling"] = bench_buckling(ctx, stream)
        print(f"# buckling: {json.dumps(out['buckling'])}", file=sys.stderr, flush=True)
    if "levelset" in secs:
        out["levelset"] = bench_levelset(ctx, stream)
        print(f"# level-set loop: {json.dumps(out['levelset'])}", file=sys.stderr, flush=True)
    if "small" in secs:
        out["small_solve"] = bench_small_solve(ctx, stream)
        print(f"# 24x12x12: {json.dumps(out['small_solve'])}", file=sys.stderr, flush=True)
    if "serve" in secs:
        out["serving"] = bench_serve(ctx, args)
        print(f"# serving: {json.dumps(out['serving'])}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["mixed_error_vs_oracle"] = mixed_vs_oracle(ctx, stream)
        print(f"# mixed vs oracle: {json.dumps(out['mixed_error_vs_oracle'])}", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
        print(f"# cpu baseline: {json.dumps(out['cpu_baseline'])}", file=sys.stderr, flush=True)
    afdcg.afd_context_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
