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
TRAFFIC_BYTES = 74_631_168 + 43_918_438


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


def cpu_baseline(budget_s=20.0):
    """The CPU oracle (assembled CSR, scipy) on a bounded sample of the same
    recipe: the 96x48x48 replica (1/8 of the volume); reports CSR K.u GDOF/s."""
    import scipy
    from oracle import fem
    from paper_2203_15115_amd import workloads as wl
    dims = (96, 48, 48)
    p = wl.cantilever(dims, 50, seed=1001, ell=dims[0] / 12.0, block=(8, 8, 8))
    t0 = time.perf_counter()
    K = fem.assemble(p.dims, p.rho, fem.ke_gauss())
    t_asm = time.perf_counter() - t0
    u = np.random.default_rng(0).standard_normal(p.ndof)
    y = K @ u
    reps, t0 = 0, time.perf_counter()
    while True:
        y = K @ u
        reps += 1
        if time.perf_counter() - t0 > min(budget_s, 10.0) and reps >= 3:
            break
    t = (time.perf_counter() - t0) / reps
    return {"value": round(p.ndof / t / 1e9, 4), "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"scipy CSR SpMV of the assembled K on the 96x48x48 replica of the workload "
                      f"({p.ndof} DOF, {K.nnz} nonzeros), mean of {reps} products; assembly {t_asm:.1f} s; "
                      f"scipy {scipy.__version__} SpMV is single-threaded"}


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
    t_valu = _events_time(stream, lambda: afdcg.afd_apply_K(m, afdcg.AFD_FP64, 4, U, Y), 50)
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
    """Poisson stream of cantilever requests nx x nx/2 x nx/2, nx uniform in
    {32,...,160}, 20-60% void, 1-4 RHS, to 1e-8: the continuous-batching
    server (mixed precision, 4 slots) against one-at-a-time FP64 solves in
    arrival order on the same GPU."""
    import numpy as np
    from paper_2203_15115_amd import afdcg, workloads as wl
    n = args.serve_requests
    reqs = wl.request_stream(n, rate=0.0, seed=7)
    probs = [wl.request_problem(r) for r in reqs]

    def run_server(arrivals, prec, slots):
        srv = afdcg.afd_server_create(ctx, 0, slots)
        subs = []
        t0 = time.perf_counter()
        for p, ta in zip(probs, arrivals):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.0005)
            r = afdcg.ServerRequest(p.dims, p.rho, p.fixed, p.F, block=p.block, rtol=1e-8, precision=prec)
            r.arrive = time.perf_counter() - t0
            afdcg.afd_server_submit(srv, r)
            subs.append(r)
        codes = [afdcg.afd_server_wait(srv, r.ticket, 600.0) for r in subs]
        t_end = time.perf_counter() - t0
        afdcg.afd_server_destroy(srv)
        done_rel = [r.res.t_done - r.res.t_submit + 0.0 for r in subs]
        return subs, codes, t_end, done_rel

    # saturated throughput of the batching server (all requests queued at t=0)
    _, codes, t_sat, _ = run_server([0.0] * n, afdcg.AFD_MIXED, 4)
    print(f"# serving: saturated {n} requests in {t_sat:.2f} s", file=sys.stderr, flush=True)
    rate = 0.8 * n / t_sat
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    res = {}
    for name, prec, slots in (("batched_mixed_4slots", afdcg.AFD_MIXED, 4), ("fifo_fp64_1slot", afdcg.AFD_FP64, 1)):
        subs, codes, t_end, lat = run_server(arrivals, prec, slots)
        lat = np.array(lat)
        print(f"# serving: {name} done in {t_end:.2f} s", file=sys.stderr, flush=True)
        res[name] = {"solves_per_s": round(n / t_end, 3), "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                     "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                     "ok": int(sum(c == 0 for c in codes)), "requests": n,
                     "max_rel_residual": max(s.rel_residual_true for r in subs for s in r.stats)}
    return {"workload": f"{n} Poisson-arrival requests, nx in 32..160, 1-4 RHS, rtol 1e-8",
            "saturated_solves_per_s": round(n / t_sat, 3), "arrival_rate_per_s": round(rate, 3), **res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=200, help="timed operator applies")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--sections", default="multi,mixed,serve",
                    help="extra measured sections: multi (4-RHS, VALU vs matrix cores), mixed, serve")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--apply-only", action="store_true",
                    help="only a known-size copy and the timed applies (hardware-counter runs)")
    ap.add_argument("--apply-config", default="-1:0",
                    help="with --apply-only: variant:zc of the applies (-1:0 the default; no autotuning)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
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
        u = torch.randn(p.ndof, dtype=torch.float64, device=dev)
        y = torch.empty_like(u)
        for _ in range(2000 + args.reps):  # 2000 warm-up launches (steady clocks), then the counted ones
            afdcg.afd_apply_K(mesh, afdcg.AFD_FP64, 1, u, y)
        torch.cuda.synchronize()
        print(json.dumps({"apply_only": True, "copy_bytes": 2 * a.numel() * 8, "reps": args.reps, "warmup": 2000,
                          "apply_config": {"variant": v, "zc": zc}}), flush=True)
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

    u = torch.randn(p.ndof, dtype=torch.float64, device=dev)
    y = torch.empty_like(u)
    t_apply, apply_launch = time_applies(afdcg.AFD_FP64, u, y)
    gdofs = p.ndof / t_apply / 1e9
    alg = matvec_algorithmic_bytes(p.dims)
    achieved = alg / t_apply / 1e9
    print(f"# apply: {t_apply * 1e6:.1f} us/launch, {gdofs:.1f} GDOF/s, {achieved:.0f} GB/s algorithmic",
          file=sys.stderr, flush=True)
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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
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
    # the opt-in coarse solve over FP32 copies of the FP64 factor's solve
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
    if "serve" in secs:
        out["serving"] = bench_serve(ctx, args)
        print(f"# serving: {json.dumps(out['serving'])}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    afdcg.afd_context_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
