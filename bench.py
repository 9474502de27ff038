"""Benchmark: FP64 PISO steps/s on the 1,053,696-tet Kuhn cube (56^3 hexes, node jitter 0.15h) set up
as a channel (parabolic inlet at x=0, Windkessel RCR outlet at x=1, no-slip walls), two correctors,
PCG tol 1e-8, BiCGStab momentum.  Also reports per-operator throughput on the same mesh in FP64 and
FP32 (faces/s and fraction of the 8 TB/s HBM roofline), the roofline of the dominant kernel measured
live with HIP events, and the CPU oracle timed on the host on a bounded sample.

Prints one JSON line.  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PISO steps/s & faces/s/operator at 1M cells FP64 (% HBM peak); adjoint/fwd ratio"
HBM_PEAK_GBS = 8000.0

# HBM-side bytes per launch of k_pcg_spmv on this workload from two rocprofv3 --pmc runs (TCC
# FETCH_SIZE and WRITE_SIZE medians in KiB, scaled by what the counters read for a 256 MiB device
# copy), valid only for the kernel source they were taken with.
PCG_SPMV_COUNTERS = {"source": "paper_2603_15920_amd/csrc/krylov.hip",
                     "sha256": "a77a33155fd0c286988320d66c063f5ae3770182a823c829edbe778cf41763f8",
                     "fetch_kib": 33814.4, "write_kib": 16472.4, "fetch_scale": 2.0, "write_scale": 1.0}


def counter_traffic(c):
    """Scaled counter bytes per launch, or None once the kernel source differs from the one measured."""
    import hashlib
    try:
        h = hashlib.sha256(open(os.path.join(ROOT, c["source"]), "rb").read()).hexdigest()
    except OSError:
        return None
    if h != c["sha256"]:
        return None
    return int(round(1024 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])))


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def channel_setup(mg, n=56, seed=2603002):
    m = mg.kuhn_cube(n, jitter=0.15, patches="channel", seed=seed)
    Fi = m.n_internal_faces
    import numpy as np
    Ub = np.zeros((m.n_boundary_faces, 3))
    inl = m.patch("inlet")
    c = m.Cf[inl.start:inl.start + inl.size]
    Ub[inl.start - Fi:inl.start - Fi + inl.size, 0] = 16 * c[:, 1] * (1 - c[:, 1]) * c[:, 2] * (1 - c[:, 2])
    q_in = -float((Ub[inl.start - Fi:inl.start - Fi + inl.size] * m.Sf[inl.start:inl.start + inl.size]).sum())
    # nominal RCR for a single outlet: Rd = 1/Q, Rp = Rd/9, C = tau/Rd with tau = 0.1
    Rd = 1.0 / q_in
    wk = (Rd / 9.0, 0.1 / Rd, Rd)
    return m, Ub, wk, q_in


# algorithmic bytes per launch (each input read once, each output written once; int32 indices)
def op_bytes(op, nfi, nfb, nc, fp):
    i4 = 4
    if op == "grad":
        return nfi * (2 * i4 + fp + 3 * fp) + nfb * (i4 + 3 * fp + fp) + nc * (fp + fp + 3 * fp)
    if op == "laplacian":
        return nfi * (2 * i4 + fp + 3 * fp + fp) + nfb * (i4 + fp + fp) + nc * (fp + 3 * fp + fp)
    if op == "div_upwind_vec":
        return nfi * (2 * i4 + fp) + nfb * (i4 + fp + 3 * fp) + nc * (3 * fp + 3 * fp)
    if op == "spmv":
        return nfi * (2 * i4 + fp + fp) + nc * 3 * fp
    if op == "spmv_sym":
        return nfi * (2 * i4 + fp) + nc * 3 * fp
    if op == "interp":
        return nfi * (2 * i4 + fp + fp) + nfb * (i4 + fp + fp) + nc * fp
    if op == "pcg_spmv":
        # the PCG product with its fused direction update p_k = z + beta p_(k-1): per face O, N and the
        # symmetric coefficient; per cell diag, z and p_(k-1) read, p_k and q = K p_k written
        return nfi * (2 * i4 + fp) + nc * 5 * fp
    raise KeyError(op)


class HipTimer:
    """HIP events created with hipEventDisableSystemFence (timing only: no cache write-back around the
    timed work), recorded on the given stream."""

    def __init__(self, stream):
        import ctypes
        self.C = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.stream = ctypes.c_void_p(stream.cuda_stream)
        self.e0, self.e1 = ctypes.c_void_p(), ctypes.c_void_p()
        for e in (self.e0, self.e1):
            assert self.hip.hipEventCreateWithFlags(ctypes.byref(e), ctypes.c_uint(0x20000000)) == 0

    def start(self):
        assert self.hip.hipEventRecord(self.e0, self.stream) == 0

    def stop_s(self):
        assert self.hip.hipEventRecord(self.e1, self.stream) == 0
        assert self.hip.hipEventSynchronize(self.e1) == 0
        ms = self.C.c_float()
        assert self.hip.hipEventElapsedTime(self.C.byref(ms), self.e0, self.e1) == 0
        return ms.value * 1e-3


def operator_sweep(B, M, m, torch, reps=30, warm_runs=True):
    """Per-operator kernel time with HIP events on the launch stream; the 256 MB Infinity Cache is
    flushed by reading a 1 GiB buffer before every timed launch (cold numbers; a read leaves no dirty
    lines to write back), warm numbers back to back."""
    import numpy as np
    from paper_2603_15920_amd import meshgen as mg
    nc, nfi, nfb = m.n_cells, m.n_internal_faces, m.n_boundary_faces
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype=dt)
    f = mg.sinusoid_field(2603012)
    phi_u = f(m.C)
    phib_u = f(m.Cf[nfi:])
    U_u = np.stack([mg.sinusoid_field(2603013 + k)(m.C) for k in range(3)], 1)
    Ub_u = np.stack([mg.sinusoid_field(2603013 + k)(m.Cf[nfi:]) for k in range(3)], 1)
    flush = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    sink = torch.empty((), dtype=torch.float32, device="cuda:0")
    out = {}
    s = torch.cuda.current_stream()
    tm = HipTimer(s)
    # reference: a plain device copy of 64 MiB (128 MiB moved), timed the same way
    src = torch.ones(1 << 23, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    cold = []
    for _ in range(reps):
        sink = flush.sum()
        tm.start()
        dst.copy_(src)
        cold.append(tm.stop_s())
    tm.start()
    for _ in range(reps):
        dst.copy_(src)
    warm = tm.stop_s() / reps
    tc = sorted(cold)[len(cold) // 2]
    out["copy_64MiB_reference"] = {"us_cold": round(tc * 1e6, 2), "us_warm": round(warm * 1e6, 2),
                                   "GBps_cold": round(2 * src.numel() * 8 / tc / 1e9, 1),
                                   "GBps_warm": round(2 * src.numel() * 8 / warm / 1e9, 1)}
    log("copy reference", out["copy_64MiB_reference"])
    del src, dst
    for dt, tag, fp in ((torch.float64, "fp64", 8), (torch.float32, "fp32", 4)):
        phi = M.to_internal(dev(phi_u, dt), B.KIND_CELL)
        phib = M.to_internal(dev(phib_u, dt), B.KIND_BFACE)
        U = M.to_internal(dev(U_u, dt), B.KIND_CELL)
        Ub = M.to_internal(dev(Ub_u, dt), B.KIND_BFACE)
        g = torch.empty((nc, 3), dtype=dt, device="cuda:0")
        B.difvm_op_grad(M.h, 1, B.BC_ALL_FIXED, phi, phib, g)
        Uf = torch.empty((nfi + nfb, 3), dtype=dt, device="cuda:0")
        B.difvm_op_interp(M.h, 3, B.BC_ALL_FIXED, U, Ub, Uf)
        # face flux F = U_f . S in internal order (built from the library's interpolation, only as input)
        S = torch.from_numpy(np.ascontiguousarray(m.Sf)).to("cuda:0", dtype=dt)
        flux = M.to_internal((M.to_user(Uf, B.KIND_FACE) * S).sum(1).contiguous(), B.KIND_FACE_FLUX)
        diag = torch.full((nc,), 6.0, dtype=dt, device="cuda:0")
        up = -torch.rand(nfi, dtype=dt, device="cuda:0")
        lo = -torch.rand(nfi, dtype=dt, device="cuda:0")
        o1 = torch.empty(nc, dtype=dt, device="cuda:0")
        o3 = torch.empty((nc, 3), dtype=dt, device="cuda:0")
        of = torch.empty(nfi + nfb, dtype=dt, device="cuda:0")
        A = B.ldu(diag, up, lo)
        As = B.ldu(diag, up)
        ops = {
            "grad": lambda: B.difvm_op_grad(M.h, 1, B.BC_ALL_FIXED, phi, phib, o3),
            "laplacian": lambda: B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, None, phi, g, phib, o1),
            "div_upwind_vec": lambda: B.difvm_op_div(M.h, B.SCHEME_UPWIND, 3, B.BC_ALL_FIXED, flux, U, Ub, o3),
            "spmv": lambda: B.difvm_ldu_spmv(M.h, 1, 0, A, phi, o1),
            "spmv_sym": lambda: B.difvm_ldu_spmv(M.h, 1, 0, As, phi, o1),
            "interp": lambda: B.difvm_op_interp(M.h, 1, B.BC_ALL_FIXED, phi, phib, of),
        }
        for name, fn in ops.items():
            for _ in range(5):
                fn()
            cold = []
            for _ in range(reps):
                sink = flush.sum()
                tm.start()
                fn()
                cold.append(tm.stop_s())
            warm = float("nan")
            if warm_runs:
                tm.start()
                for _ in range(reps):
                    fn()
                warm = tm.stop_s() / reps
            tc = sorted(cold)[len(cold) // 2]
            nbytes = op_bytes(name, nfi, nfb, nc, fp)
            out[f"{name}_{tag}"] = {
                "us_cold": round(tc * 1e6, 2), "us_warm": round(warm * 1e6, 2) if warm_runs else None,
                "faces_per_s": round(nfi / tc, 0), "alg_MB": round(nbytes / 1e6, 2),
                "GBps_cold": round(nbytes / tc / 1e9, 1), "frac_hbm_cold": round(nbytes / tc / 1e9 / HBM_PEAK_GBS, 3),
                "GBps_warm": round(nbytes / warm / 1e9, 1) if warm_runs else None}
            log(name, tag, out[f"{name}_{tag}"])
    del flush
    return out


def timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t, r


def graph_rate(P, torch, steps, wk, extra=16, start=None):
    """Eager against graph mode over the same window: the state (U, p, phi, capacitor pressures with
    Windkessel rows wk) is saved (or `start` is loaded), `steps` eager steps are timed, the state is
    restored, one step captures the graph, the state is restored again and the same `steps` are timed
    as replays."""
    if start is not None:
        P.set_state(*start[:3])
        for j, row in enumerate(wk):
            P.set_windkessel(j, *row, start[3][j])
    U0, p0, phi0, pc0 = P.get_state()

    def restore():
        P.set_state(U0, p0, phi0)
        for j, row in enumerate(wk):
            P.set_windkessel(j, *row, pc0[j])

    te, (ste, ite, _) = timed(torch, lambda: P.step(steps))
    restore()
    P.set_graph(True, extra)
    P.step(1)
    restore()
    r0 = P.graph_info()
    tg, (stg, itg, _) = timed(torch, lambda: P.step(steps))
    r1 = P.graph_info()
    P.set_graph(False)
    return {"steps": steps, "eager_steps_per_s": round(steps / te, 4), "graph_steps_per_s": round(steps / tg, 4),
            "speedup": round(te / tg, 4), "same_iterations": bool((ite == itg).all()), "status": [int(ste), int(stg)],
            "replays": r1[0] - r0[0], "redos": r1[1] - r0[1], "extra_iters": extra,
            "pcg_iters_per_solve": round(float(itg[:, 3:].mean()), 1)}


def precond_rate(B, M, torch, prm_kw, setup, precond, warmup, steps):
    """The main workload with another pressure preconditioner: a fresh PISO object on the same mesh from
    rest, `warmup` untimed steps, then `steps` timed steps."""
    P = B.Piso(M, B.piso_params(**prm_kw, precond=precond))
    setup(P)
    P.step(warmup)
    t, (st, it, _) = timed(torch, lambda: P.step(steps))
    P.close()
    return {"precond": precond, "steps": steps, "steps_per_s": round(steps / t, 4),
            "ms_per_step": round(1e3 * t / steps, 3), "pcg_iters_per_solve": round(float(it[:, 3:].mean()), 1),
            "status": int(st)}


def poisson_run(B, mg, torch, ctx, sizes=(12, 18, 25, 56)):
    """The paper's 3D Poisson verification workload (manufactured solution on jittered Kuhn cubes of
    10,368 / 34,992 / 93,750 cells, plus the 1,053,696-cell cube): Dirichlet data from the exact field,
    over-relaxed correction from the exact gradient, Jacobi-PCG to 1e-12.  Times assembly + solve and
    reports the L2 error against the exact field and its order between sizes."""
    import math
    import numpy as np
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    out = []
    for n in sizes:
        m = mg.kuhn_cube(n, jitter=0.15, patches="walls", seed=2603007 if n != 56 else 2603002)
        M = B.Mesh(ctx, m)
        B.difvm_tune(M.h, None)
        phib = M.to_internal(dev(mg.poisson_mms_solution(m.Cf[m.n_internal_faces:])), B.KIND_BFACE)
        g = M.to_internal(dev(mg.poisson_mms_gradient(m.C)), B.KIND_CELL)
        src = M.to_internal(dev(m.V * mg.poisson_mms_source(m.C)), B.KIND_CELL)
        e = lambda k: torch.empty(k, dtype=torch.float64, device="cuda:0")
        d, u, rbc, lap0, zero, x = e(m.n_cells), e(m.n_internal_faces), e(m.n_cells), e(m.n_cells), e(m.n_cells), e(m.n_cells)
        zero.zero_()
        A = B.ldu(d, u)

        def solve():
            B.difvm_ldu_assemble_laplace(M.h, B.BC_ALL_FIXED, None, phib, A, rbc)
            B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, None, zero, g, phib, lap0)
            torch.sub(lap0, src, out=lap0)
            x.zero_()
            return B.difvm_solve_pcg(M.h, A, lap0, x, 1e-12, 20000)
        solve()
        t, (st, it, res) = timed(torch, solve)
        phi = M.to_user(x, B.KIND_CELL).cpu().numpy()
        err = phi - mg.poisson_mms_solution(m.C)
        l2 = math.sqrt((m.V * err * err).sum() / m.V.sum())
        run = {"cells": m.n_cells, "pcg_iters": it, "status": st, "solve_ms": round(1e3 * t, 3),
               "us_per_iteration": round(1e6 * t / max(it, 1), 2), "l2_error": l2}
        # the same system with the AMG preconditioner (hierarchy built once, outside the timing)
        ts = time.perf_counter()
        amg = B.difvm_amg_create(M.h, A)
        setup_s = time.perf_counter() - ts

        def solve_amg():
            x.zero_()
            return B.difvm_solve_pcg_amg(amg, A, lap0, x, 1e-12, 500)
        solve_amg()
        ta, (sta, ita, _) = timed(torch, solve_amg)
        phia = M.to_user(x, B.KIND_CELL).cpu().numpy()
        run["amg"] = {"pcg_iters": ita, "status": sta, "solve_ms": round(1e3 * ta, 3), "setup_s": round(setup_s, 3),
                      "levels": B.difvm_amg_levels(amg),
                      "max_rel_diff_to_jacobi": float(np.abs(phia - phi).max() / np.abs(phi).max())}
        B.difvm_amg_destroy(amg)
        out.append(run)
        M.close()
    for a, b in zip(out, out[1:]):
        b["order"] = round(math.log(a["l2_error"] / b["l2_error"]) / math.log((b["cells"] / a["cells"]) ** (1 / 3)), 3)
    return {"workload": "manufactured 3D Poisson solution, jittered Kuhn cubes, exact-gradient correction, "
                        "PCG tol 1e-12 (Jacobi; 'amg': the same solve with the AMG preconditioner)", "runs": out}


def tube_run(B, mg, torch, ctx, steps, precond="amg"):
    """The full PISO configuration on the straight tube (2,000,640 tets, L/D 10, parabolic inlet at
    Re 500, p = 0 outlet, nu 1e-3, dt 1e-3, 2 correctors, PCG tol 1e-8), from rest: the first step
    untimed, then `steps` timed steps (graph mode off, tuned launch shapes)."""
    import numpy as np
    t0 = time.time()
    m = mg.tube()
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("inlet")
    Ub[p.start - Fi:p.start - Fi + p.size] = mg.parabolic_inlet(m.Cf[p.start:p.start + p.size], (0, 0, 0), 0.5, 1.0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    M = B.Mesh(ctx, m)
    B.difvm_tune(M.h, None)
    P = B.Piso(M, B.piso_params(1e-3, 1e-3, tol_p=1e-8, tol_u=1e-8, maxit_p=20000, maxit_u=2000, precond=precond))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
    log(f"tube: {m.n_cells} cells ready ({time.time() - t0:.1f}s)")
    P.step(1)
    t, (st, it, _) = timed(torch, lambda: P.step(steps))
    out = {"workload": f"tube {m.n_cells} tets, L/D 10, Re 500, p = 0 outlet, nu 1e-3, dt 1e-3, 2 correctors, "
                       f"PCG tol 1e-8 ({precond} preconditioner), steps 2-{steps + 1} from rest",
           "cells": m.n_cells, "steps": steps, "steps_per_s": round(steps / t, 4),
           "cell_steps_per_s": round(steps * m.n_cells / t, 0), "pcg_iters_per_solve": round(float(it[:, 3:].mean()), 1),
           "status": int(st)}
    P.close()
    M.close()
    return out


def halo_run(B, mg, torch, ctx, n_parts=8, part=3, reps=50):
    """The part of a single-mesh multi-GPU run that one GPU can show: the 2,000,640-tet tube split into
    n_parts RCM slabs; on one interior slab (one GPU's share) the pack and unpack kernels of one halo
    exchange (scalar and 3-vector rows) and the operators on the slab's cells plus ghosts, all timed
    with HIP events (average over reps back-to-back launches, warm).  The transfer between GPUs is not
    run (one GPU); its volume is reported."""
    import numpy as np
    t0 = time.time()
    m = mg.tube()
    Pt = B.Partition(m, n_parts)
    pm = B.PartMesh(ctx, Pt, part)
    info = pm.part
    log(f"halo: {n_parts} slabs of the {m.n_cells}-cell tube ready ({time.time() - t0:.1f}s)", info)
    nl = pm.info["n_cells"]
    tm = HipTimer(torch.cuda.current_stream())
    f64 = dict(dtype=torch.float64, device="cuda:0")

    def avg_us(fn):
        fn()
        tm.start()
        for _ in range(reps):
            fn()
        return round(tm.stop_s() / reps * 1e6, 2)

    out = {"workload": f"tube {m.n_cells} tets in {n_parts} RCM slabs; slab {part} (interior)",
           "owned_cells": info["n_owned"], "ghost_cells": info["n_ghost"], "sent_rows": info["n_send"],
           "neighbour_slabs": info["n_neighbours"], "local_internal_faces": info["n_internal_faces"],
           "exchange_bytes_scalar_f64": 8 * info["n_ghost"], "exchange_bytes_vector_f64": 24 * info["n_ghost"]}
    for ncomp, tag in ((1, "scalar"), (3, "vector")):
        x = torch.rand((nl, ncomp) if ncomp > 1 else nl, **f64)
        sb = torch.empty((info["n_send"], ncomp) if ncomp > 1 else info["n_send"], **f64)
        rb = torch.rand((info["n_ghost"], ncomp) if ncomp > 1 else info["n_ghost"], **f64)
        out[f"pack_{tag}_us"] = avg_us(lambda: pm.pack(x, sb))
        out[f"unpack_{tag}_us"] = avg_us(lambda: pm.unpack(rb, x))
    phi = torch.rand(nl, **f64)
    phib = torch.rand(info["n_boundary_faces"], **f64)
    g = torch.empty((nl, 3), **f64)
    o1 = torch.empty(nl, **f64)
    out["grad_us"] = avg_us(lambda: B.difvm_op_grad(pm.h, 1, B.BC_ALL_FIXED, phi, phib, g))
    out["laplacian_us"] = avg_us(lambda: B.difvm_op_laplacian(pm.h, B.BC_ALL_FIXED, None, phi, g, phib, o1))
    A = B.ldu(torch.full((nl,), 6.0, **f64), -torch.rand(info["n_internal_faces"], **f64))
    out["spmv_sym_us"] = avg_us(lambda: B.difvm_ldu_spmv(pm.h, 1, 0, A, phi, o1))
    pm.close()
    Pt.close()
    return out


def small_case(B, mg, torch, ctx, steps=50, precond="amg"):
    """The small PISO case (lid-driven cavity, 2048 jittered triangle prisms, Re 100, nu 0.01,
    dt 1e-3): launch-bound, so eager stepping against graph mode."""
    import numpy as np
    m = mg.cavity()
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("lid")
    Ub[p.start - m.n_internal_faces:p.start - m.n_internal_faces + p.size, 0] = 1.0
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    out = {"workload": f"cavity {m.n_cells} prisms, nu 0.01, dt 1e-3, 2 correctors, tol 1e-8 ({precond} preconditioner)",
           "cells": m.n_cells}
    M = B.Mesh(ctx, m)
    for mode in ("eager", "graph"):
        P = B.Piso(M, B.piso_params(0.01, 1e-3, precond=precond))
        P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
        P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
        if mode == "graph":
            P.set_graph(True, 16)
        P.step(3)
        t, (st, it, _) = timed(torch, lambda: P.step(steps))
        out[f"{mode}_steps_per_s"] = round(steps / t, 2)
        out[f"{mode}_status"] = int(st)
        if mode == "graph":
            out["graph_replays"], out["graph_redos"], _ = P.graph_info()
        P.close()
    out["pcg_iters_per_solve"] = round(float(it[:, 3:].mean()), 1)
    out["graph_speedup"] = round(out["graph_steps_per_s"] / out["eager_steps_per_s"], 3)
    return out


def adjoint_window(B, mg, torch, ctx, steps, every, spinup=50, precond="amg"):
    """Differentiated form on the Y-bifurcation (~400k tets, 3 Windkessel outlets, nu 1e-3, dt 1e-3):
    after a short spin-up from rest, the plain forward, the recorded forward (checkpoints every
    `every` steps) and the reverse sweep (recomputation of each checkpoint segment plus its adjoint
    steps) over the same `steps`-step window, tolerances 1e-8."""
    import numpy as np
    t0 = time.time()
    m = mg.ybif(h=0.0519)
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("inlet")
    s = slice(p.start - m.n_internal_faces, p.start - m.n_internal_faces + p.size)
    Ub[s] = mg.parabolic_inlet(m.Cf[p.start:p.start + p.size], (0.0, 0.0, 0.0), 0.5, 1.0)
    wk = mg.windkessel_nominal(m, mg.inlet_flow(m, Ub))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    M = B.Mesh(ctx, m)
    P = B.Piso(M, B.piso_params(1e-3, 1e-3, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=5000, maxit_u=1000,
                                precond=precond))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    for j, row in enumerate(wk):
        P.set_windkessel(j, *row, 0.0)
    P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
    P.step(spinup)
    log(f"adjoint: ybif {m.n_cells} cells ready ({time.time() - t0:.1f}s)")
    U0, p0, phi0, pc0 = P.get_state()
    t_fwd, (st, it, _) = timed(torch, lambda: P.step(steps))
    P.set_state(U0, p0, phi0)
    for j, row in enumerate(wk):
        P.set_windkessel(j, *row, pc0[j])
    T = B.difvm_tape_create(P.h, steps, every)
    t_rec, (st_r, _) = timed(torch, lambda: B.difvm_piso_forward_record(P.h, T, steps))
    rng = np.random.default_rng(2603024)
    gU, gp, gphi = (torch.empty_like(U0), torch.empty_like(p0), torch.empty_like(phi0))
    cot = [dev(rng.standard_normal((m.n_cells, 3))), dev(rng.standard_normal(m.n_cells)), dev(rng.standard_normal(m.n_faces)),
           rng.standard_normal(len(wk))]
    t_adj, (st_a, gpc, gwk) = timed(torch, lambda: B.difvm_piso_adjoint(P.h, T, *cot, 1e-8, gU, gp, gphi, len(wk)))
    # a second sweep on the same tape recomputes every segment (the first reverses the window's last
    # segment from the forward record's own step records): the eager reference for the graph sweeps
    t_adj2, _ = timed(torch, lambda: B.difvm_piso_adjoint(P.h, T, *cot, 1e-8, gU, gp, gphi, len(wk)))
    # the same reverse sweep with its segments replayed as graphs (the first full segment captures)
    gU_e = gU.clone()
    B.difvm_tape_set_graph(T, True, 16)
    t_adj_g1, (st_g1, _, _) = timed(torch, lambda: B.difvm_piso_adjoint(P.h, T, *cot, 1e-8, gU, gp, gphi, len(wk)))
    t_adj_g, (st_g, _, _) = timed(torch, lambda: B.difvm_piso_adjoint(P.h, T, *cot, 1e-8, gU, gp, gphi, len(wk)))
    g_info = B.difvm_tape_graph_info(T)
    same = bool(torch.equal(gU, gU_e))
    B.difvm_tape_destroy(T)
    return {"workload": f"Y-bifurcation {m.n_cells} tets, 3 RCR outlets, nu 1e-3, dt 1e-3, {spinup}-step spin-up, "
                        f"{steps}-step window, checkpoint every {every}, tol 1e-8 ({precond} preconditioner)",
            "cells": m.n_cells, "steps": steps, "ckpt_every": every,
            "forward_steps_per_s": round(steps / t_fwd, 3), "record_steps_per_s": round(steps / t_rec, 3),
            "adjoint_steps_per_s": round(steps / t_adj, 3), "adjoint_over_forward": round(t_adj / t_fwd, 3),
            "record_over_forward": round(t_rec / t_fwd, 3), "pcg_iters_per_solve": round(float(it[:, 3:].mean()), 1),
            "resweep_steps_per_s": round(steps / t_adj2, 3),
            "graph_sweep": {"first_sweep_steps_per_s": round(steps / t_adj_g1, 3),
                            "replayed_sweep_steps_per_s": round(steps / t_adj_g, 3),
                            "speedup_vs_eager": round(t_adj2 / t_adj_g, 3), "bitwise_equal_to_eager": same,
                            "replays_redos_captures": list(g_info), "status": [int(st_g1), int(st_g)]},
            "status": [int(st), int(st_r), int(st_a)]}


def batch_run(B, mg, torch, ctx, n_members, steps, adj_steps, precond="amg"):
    """Batched form: n_members seeded meshes of uneven size packed block-diagonally into one mesh of
    segments, each with its own viscosity and Windkessel; steps/s of the batch against the same members
    advanced one after another as separate meshes, and a checkpointed window of adj_steps through the
    batch (checkpoint every adj_steps/2)."""
    import numpy as np
    t0 = time.time()
    mem = mg.batch_members(n_members)
    Pm, starts = mg.pack([d["mesh"] for d in mem])
    log(f"batch: {n_members} members, {Pm.n_cells} cells ({time.time() - t0:.1f}s)")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    prm = dict(dt=1e-3, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=5000, maxit_u=1000)

    def setup(mesh, Ub, wk, nus, seg=None):
        M = B.Mesh(ctx, mesh, seg_cell_start=seg)
        P = B.Piso(M, B.piso_params(float(nus[0]), **prm, precond=precond))
        if seg is not None:
            P.set_viscosity(nus)
        P.set_boundary(dev(Ub), dev(np.zeros(mesh.n_boundary_faces)))
        for j, row in enumerate(wk):
            P.set_windkessel(j, *row, 0.0)
        P.set_state(dev(np.zeros((mesh.n_cells, 3))), dev(np.zeros(mesh.n_cells)), None)
        return M, P

    Mb, Pb = setup(Pm, np.concatenate([d["Ub"] for d in mem]), np.concatenate([d["wk"] for d in mem]),
                   np.array([d["nu"] for d in mem]), starts)
    B.difvm_tune(Mb.h, None)
    log(f"batch: device mesh ready ({time.time() - t0:.1f}s)")
    Pb.step(2)
    t_b, (st, it, _) = timed(torch, lambda: Pb.step(steps))
    seg_it, _, seg_st = Pb.segment_stats()
    gr = graph_rate(Pb, torch, steps, np.concatenate([d["wk"] for d in mem]))
    t_seq = 0.0
    for d in mem:
        M, P = setup(d["mesh"], d["Ub"], d["wk"], [d["nu"]])
        P.step(2)
        dt_, _ = timed(torch, lambda: P.step(steps))
        t_seq += dt_
        P.close()
        M.close()
    out = {"workload": f"{n_members} seeded members (even: tubes, odd: box channels), sizes log-uniform in "
                       f"[2e4, 3e5] cells, Re in [100, 800], one RCR each, dt 1e-3, 2 correctors, tol 1e-8 "
                       f"({precond} preconditioner)",
           "members": n_members, "cells": Pm.n_cells, "steps": steps,
           "batch_steps_per_s": round(steps / t_b, 3),
           "batch_cell_steps_per_s": round(steps * Pm.n_cells / t_b, 0),
           "sequential_steps_per_s": round(steps / t_seq, 3),
           "speedup_vs_sequential": round(t_seq / t_b, 3),
           "batch_graph": gr,
           "pcg_iters_max_member": int(seg_it[:, 3:].max()), "pcg_iters_min_member": int(seg_it[:, 3:].min()),
           "status": int(st)}
    if adj_steps > 0:
        T = B.difvm_tape_create(Pb.h, adj_steps, max(1, adj_steps // 2))
        t_rec, _ = timed(torch, lambda: B.difvm_piso_forward_record(Pb.h, T, adj_steps))
        rng = np.random.default_rng(2603025)
        U0 = torch.empty((Pm.n_cells, 3), dtype=torch.float64, device="cuda:0")
        gU, gp, gphi = U0, torch.empty(Pm.n_cells, dtype=torch.float64, device="cuda:0"), \
            torch.empty(Pm.n_faces, dtype=torch.float64, device="cuda:0")
        cot = [dev(rng.standard_normal((Pm.n_cells, 3))), dev(rng.standard_normal(Pm.n_cells)),
               dev(rng.standard_normal(Pm.n_faces)), rng.standard_normal(n_members)]
        t_adj, (st_a, _, _) = timed(torch, lambda: B.difvm_piso_adjoint(Pb.h, T, *cot, 1e-8, gU, gp, gphi, n_members))
        B.difvm_tape_destroy(T)
        out.update({"adjoint_window_steps": adj_steps, "record_steps_per_s": round(adj_steps / t_rec, 3),
                    "adjoint_steps_per_s": round(adj_steps / t_adj, 3), "adjoint_status": int(st_a)})
    Pb.close()
    Mb.close()
    return out


def oracle_operator_times(O, m, reps=5):
    """The oracle's FP64 face operators on the operator sweep's inputs (same fields and seeds), one
    core, median of `reps` calls, with internal faces per second."""
    import numpy as np
    from paper_2603_15920_amd import meshgen as mg
    nfi = m.n_internal_faces
    f = mg.sinusoid_field(2603012)
    phi, phib = f(m.C), f(m.Cf[nfi:])
    U = np.stack([mg.sinusoid_field(2603013 + k)(m.C) for k in range(3)], 1)
    Ub = np.stack([mg.sinusoid_field(2603013 + k)(m.Cf[nfi:]) for k in range(3)], 1)
    g = O.grad(m, phi, phib)
    flux = np.einsum("fi,fi->f", O.interp(m, U, Ub), m.Sf)
    rng = np.random.default_rng(5)
    d, up, lo = np.full(m.n_cells, 6.0), -rng.random(nfi), -rng.random(nfi)
    calls = {"grad": lambda: O.grad(m, phi, phib),
             "laplacian": lambda: O.laplacian(m, phi, g, phib),
             "div_upwind_vec": lambda: O.div(m, flux, U, Ub, scheme=O.SCHEME_UPWIND),
             "spmv": lambda: O.spmv(m, d, up, lo, phi),
             "spmv_sym": lambda: O.spmv(m, d, up, up, phi),
             "interp": lambda: O.interp(m, phi, phib)}
    out = {}
    for name, fn in calls.items():
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[len(ts) // 2]
        out[name] = {"ms": round(t * 1e3, 2), "faces_per_s": round(nfi / t, 1)}
    return out


def cpu_info():
    """CPU model from lscpu (else /proc/cpuinfo) and the host threads available to this process."""
    model = ""
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model:
        return f"{model} ({len(os.sched_getaffinity(0))} threads available)"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model or platform.processor()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=56, help="hexes per side of the Kuhn cube")
    ap.add_argument("--no-ops", action="store_true", help="skip the per-operator sweep")
    ap.add_argument("--ops-only", action="store_true",
                    help="only the per-operator sweep (prints its own JSON line, not the benchmark line)")
    ap.add_argument("--ops-reps", type=int, default=30, help="cold (and warm) launches per operator")
    ap.add_argument("--ops-warm", type=int, default=1, help="with --ops-only: 0 times cold launches only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiated-window measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-mesh batch measurement")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (no autotuning)")
    ap.add_argument("--no-poisson", action="store_true", help="skip the Poisson verification workload")
    ap.add_argument("--no-tube", action="store_true", help="skip the 2M-cell tube PISO run")
    ap.add_argument("--tube-steps", type=int, default=50)
    ap.add_argument("--no-halo", action="store_true", help="skip the slab-partition halo measurement")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-mode measurements")
    ap.add_argument("--graph-extra", type=str, default="16",
                    help="graph mode's iteration margin per solve; several, comma-separated, time one window each")
    ap.add_argument("--precond", choices=["jacobi", "amg"], default="amg",
                    help="pressure preconditioner of the timed PISO steps")
    ap.add_argument("--no-other", action="store_true", help="skip the run with the other pressure preconditioner")
    ap.add_argument("--adj-steps", type=int, default=100)
    ap.add_argument("--adj-every", type=int, default=10)
    ap.add_argument("--batch-members", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-adj-steps", type=int, default=20)
    ap.add_argument("--prof-every", type=int, default=16,
                    help="time every n-th launch of each PCG kernel with HIP events in the timed region")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library computes on a single GPU "
              "(the slab partition and halo kernels show one GPU's share of a multi-GPU run).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_15920_amd import binding as B
    from paper_2603_15920_amd import meshgen as mg

    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_mib} MiB read + {args.copy_mib} MiB written")
        del src, dst

    t0 = time.time()
    m, Ub, wk, q_in = channel_setup(mg, args.n)
    nc, nfi, nfb = m.n_cells, m.n_internal_faces, m.n_boundary_faces
    log(f"mesh {nc} cells {nfi} internal faces {nfb} boundary faces ({time.time() - t0:.1f}s)")
    nu, dt = 0.005, 1e-3   # Re = Umax L / nu = 200, diffusion number nu dt / h^2 = 0.016
    ctx = B.Context(0)
    M = B.Mesh(ctx, m)
    log("device mesh", M.info)
    if args.ops_only:
        # operator timings alone (for a kernel trace: cold launches only unless --ops-warm)
        if not args.no_tune:
            B.difvm_tune(M.h, None)
        ops = operator_sweep(B, M, m, torch, reps=args.ops_reps, warm_runs=args.ops_warm)
        print(json.dumps({"operators": ops, "cells": nc, "internal_faces": nfi, "boundary_faces": nfb,
                          "reps": args.ops_reps, "tuned_launch": {name: B.difvm_mesh_get_launch(M.h, k)
                                                                  for k, name in enumerate(B.TUNE_KNOBS)}}),
              flush=True)
        return
    prm_kw = dict(nu=nu, dt=dt, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=5000, maxit_u=1000)
    P = B.Piso(M, B.piso_params(**prm_kw, precond=args.precond))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    U0, p0 = np.zeros((nc, 3)), np.zeros(nc)

    def setup(Pp):
        Pp.set_boundary(dev(Ub), dev(np.zeros(nfb)))
        Pp.set_windkessel(0, *wk, 0.0)
        Pp.set_state(dev(U0), dev(p0), None)
    setup(P)
    torch.cuda.synchronize()
    tuned = None
    if not args.no_tune:
        tt = time.time()
        B.difvm_tune(M.h, None)
        tuned = {name: B.difvm_mesh_get_launch(M.h, k) for k, name in enumerate(B.TUNE_KNOBS)}
        log(f"tuned launch shapes ({time.time() - tt:.2f}s)", tuned)

    first_step_s = None
    for k in range(args.warmup):
        ts = time.time()
        st, it, res = P.step(1)
        torch.cuda.synchronize()
        if k == 0:
            first_step_s = time.time() - ts
            first_iters = it[0].tolist()
        log(f"warmup step {k}: {time.time() - ts:.3f}s iters {it[0].tolist()} status {st}")

    # the state the timed region starts from (the graph-mode window and the CPU oracle start from it)
    U_s, p_s, phi_s, pc_s = P.get_state()
    start_dev = (U_s.clone(), p_s.clone(), phi_s.clone(), np.array(pc_s, dtype=np.float64))
    state0 = None
    if not args.no_cpu:
        state0 = (U_s.cpu().numpy(), p_s.cpu().numpy(), phi_s.cpu().numpy(), np.array(pc_s, dtype=np.float64))
    del U_s, p_s, phi_s
    # timed region: eager steps, HIP events around every prof_every-th launch of each PCG kernel
    B.difvm_ctx_profile(ctx.h, args.prof_every)
    B.difvm_ctx_profile_read(ctx.h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, it, res = P.step(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prof = B.difvm_ctx_profile_read(ctx.h)
    B.difvm_ctx_profile(ctx.h, 0)
    elapsed = t2 - t1
    steps_per_s = args.steps / elapsed
    log(f"timed {args.steps} steps in {elapsed:.3f}s -> {steps_per_s:.3f} steps/s; status {st}")
    log("kernel events", prof)
    pcg_iters = it[:, 3:].sum()

    # dominant kernel: the PCG matrix-vector product with its p.q reduction
    name = "pcg_spmv_dot"
    launches, total_ms = prof.get(name, (0, 0.0))  # every prof_every-th launch, HIP events
    avg_s = total_ms * 1e-3 / max(launches, 1)
    alg = op_bytes("pcg_spmv", nfi, nfb, nc, 8)
    achieved = alg / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = counter_traffic(PCG_SPMV_COUNTERS)
    roofline = {"bound": "hbm", "kernel": "k_pcg_spmv", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": alg, "avg_launch_us": round(avg_s * 1e6, 2), "timed_launches": launches,
                "timed_every": args.prof_every, "active_iterations": int(pcg_iters)}
    kernel_us = {k: round(1e3 * v[1] / max(v[0], 1), 2) for k, v in prof.items()}
    vcycle = None
    if args.precond == "amg" and "pcg_amg_vcycle" in prof:
        # the preconditioner phase as a whole: one V-cycle's algorithmic bytes (library accounting,
        # difvm_piso_precond_info) over the HIP-event time of one V-cycle (all its kernels)
        levels, vbytes = B.difvm_piso_precond_info(P.h)
        vl, vms = prof["pcg_amg_vcycle"]
        v_s = vms * 1e-3 / max(vl, 1)
        vcycle = {"bound": "hbm", "phase": "AMG V-cycle (all kernels of one application)", "levels": levels,
                  "alg_bytes_per_vcycle": int(vbytes), "avg_vcycle_us": round(v_s * 1e6, 2),
                  "achieved": round(vbytes / v_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(vbytes / v_s / 1e9 / HBM_PEAK_GBS, 4), "timed_vcycles": vl}
        log("v-cycle roofline", vcycle)

    # per-phase breakdown of the step: 10 more eager steps after the timed region with only the phase
    # events on (HIP events on the stream around each phase; kernel events off)
    nph = 10
    B.difvm_ctx_profile_phases(ctx.h, 1)
    B.difvm_ctx_profile_read(ctx.h)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    P.step(nph)
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    phd = B.difvm_ctx_profile_read(ctx.h)
    B.difvm_ctx_profile_phases(ctx.h, 0)
    phases = {k[len("step: "):].replace(" ", "_") + "_ms": round(v[1] / nph, 3)
              for k, v in phd.items() if k.startswith("step: ")}
    phase_breakdown = {"steps": nph, "ms_per_step": round(1e3 * (tp1 - tp0) / nph, 3), **phases,
                       "outside_phases_ms": round(1e3 * (tp1 - tp0) / nph - sum(phases.values()), 3),
                       "note": "per step, summed over the correctors; the pressure solve includes the GPU's idle "
                               "time while the host polls the solver"}
    log("phase breakdown", phase_breakdown)

    # passive scalar carried by the flow of the last step (D = 1e-4, zeroGradient walls and outlet)
    scalar = None
    if not args.no_poisson:
        c = torch.from_numpy(np.exp(-((m.C - np.array([0.3, 0.5, 0.5])) ** 2).sum(1) / 0.05)).to("cuda:0")
        cb = torch.zeros(nfb, dtype=torch.float64, device="cuda:0")
        P.transport_scalar(1e-4, B.BC_U, cb, c)
        ts_, (sts, its, _) = timed(torch, lambda: P.transport_scalar(1e-4, B.BC_U, cb, c))
        scalar = {"workload": "passive scalar blob in the channel's last flux, D 1e-4, implicit Euler, upwind, "
                              "BiCGStab tol 1e-8", "cells": nc, "step_ms": round(1e3 * ts_, 3), "bicgstab_iters": its,
                  "status": sts}
        log("scalar", scalar)

    alt = None
    if not args.no_other:
        other = "jacobi" if args.precond == "amg" else "amg"
        alt = precond_rate(B, M, torch, prm_kw, setup, other, args.warmup, min(args.steps, 5))
        log("other preconditioner", alt)

    graph = None
    small = None
    if not args.no_graph:
        extras = [int(e) for e in args.graph_extra.split(",")]
        for e in extras:
            # the headline's own window (same start state, same steps), eagerly and as replays
            graph = graph_rate(P, torch, args.steps, [wk], extra=e, start=start_dev)
            log("graph mode", graph)
        small = small_case(B, mg, torch, ctx, precond=args.precond)
        log("small case", small)

    tube = None
    if not args.no_tube:
        tube = tube_run(B, mg, torch, ctx, args.tube_steps, precond=args.precond)
        log("tube", tube)
    halo = None
    if not args.no_halo:
        halo = halo_run(B, mg, torch, ctx)
        log("halo", halo)
    poisson = None
    if not args.no_poisson:
        poisson = poisson_run(B, mg, torch, ctx)
        log("poisson", poisson)
    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_window(B, mg, torch, ctx, args.adj_steps, args.adj_every, precond=args.precond)
        log("adjoint window", adjoint)
    batched = None
    if not args.no_batch:
        batched = batch_run(B, mg, torch, ctx, args.batch_members, args.batch_steps, args.batch_adj_steps,
                            precond=args.precond)
        log("batched", batched)

    ops = None
    if not args.no_ops:
        ops = operator_sweep(B, M, m, torch)

    cpu = None
    if not args.no_cpu:
        from oracle import build as OB
        from oracle import oracle as O
        oprm = O.piso_params(nu, dt, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=5000, maxit_u=1000)
        legs = {}
        for variant in ("omp", "serial"):
            O.use_threads(variant == "omp")
            nthr = O.threads()
            tc = time.time()
            r = O.piso_run(m, oprm, state0[0], state0[1], state0[2], Ub, np.zeros(nfb), wk=np.array([wk]),
                           pc=state0[3], nsteps=1)
            legs[variant] = {"seconds": round(time.time() - tc, 3), "threads": nthr, "iters": r[4][0].tolist(),
                             "status": int(r[6])}
            log(f"cpu oracle ({variant})", legs[variant])
        O.use_threads(False)
        ops_cpu = oracle_operator_times(O, m)
        log("cpu oracle operators (one core)", ops_cpu)
        om = legs["omp"]
        cpu = {"value": round(1.0 / om["seconds"], 5), "unit": "steps/s", "cores": om["threads"], "kind": "oracle",
               "sample": f"one PISO step of the oracle from the GPU's state at the start of the timed region (step "
                         f"{args.warmup + 1} of the run: same mesh, physics and tolerances); the oracle's pressure "
                         f"CG is Jacobi-preconditioned (it has no AMG), so it iterates more: oracle iterations "
                         f"{om['iters']} against the GPU's {it[0].tolist()} on that step",
               "seconds": om["seconds"],
               "single_core": {"value": round(1.0 / legs["serial"]["seconds"], 5), "cores": 1,
                               "seconds": legs["serial"]["seconds"]},
               "threading": "OpenMP over the Krylov kernels (LDU product and dot products: contiguous face and "
                            "cell ranges per thread, partial sums added in thread order)",
               "operators_single_core": {"sample": "the oracle's FP64 face operators on the operator workload's "
                                                   "inputs, median of 5 calls", **ops_cpu},
               "cpu_model": cpu_info(), "compiler": OB.compiler_version(), "flags": " ".join(OB.FLAGS_SHOWN)}
        log("cpu oracle", cpu)

    line = {
        "metric": METRIC, "value": round(steps_per_s, 4), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"PISO channel on the Kuhn cube {args.n}^3 hexes -> {nc} tets (jitter 0.15h), "
                               "parabolic inlet, Windkessel outlet, Re 200, dt 1e-3, 2 correctors, PCG tol 1e-8 "
                               f"({args.precond} preconditioner)",
                   "cells": nc, "internal_faces": nfi, "boundary_faces": nfb, "nu": nu, "dt": dt, "n_corr": 2,
                   "tol_p": 1e-8, "tol_u": 1e-8, "pressure_preconditioner": args.precond},
        "roofline": roofline,
        "vcycle_roofline": vcycle,
        "cpu_baseline": cpu, "phase_breakdown": phase_breakdown,
        "solver": {"pcg_iters_per_solve": round(float(it[:, 3:].mean()), 1),
                   "bicgstab_iters_per_component": round(float(it[:, :3].mean()), 1), "status": int(st),
                   "pressure_preconditioner": args.precond},
        "other_preconditioner": alt,
        "kernel_avg_us_timed_region": kernel_us,
        "tuned_launch": tuned,
        "graph_mode": graph,
        "small_case": small,
        "scalar_transport": scalar,
        "tube": tube,
        "halo": halo,
        "poisson": poisson,
        "adjoint": adjoint,
        "batched": batched,
        "operators": ops,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
