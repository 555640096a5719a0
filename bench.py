#!/usr/bin/env python3
"""Throughput of the mapped structured multigrid solve on one MI355X.

Headline workload: a 4097 x 4097 logical grid (16.8M unknowns) of a star-shaped domain
(conformal square->disk map composed with a radial star deformation, boundary radius
1 + sum_{k<=8} a_k cos(k theta + phi_k)), log-normal K (sigma 1, correlation length 0.1),
b ~ U(-1,1), homogeneous Dirichlet, solved from u = 0 to ||b - A u|| <= 1e-10 ||b|| in float64
(V(1,1) cycles) and with float32 V-cycles inside float64 iterative refinement.  All inputs are
synthetic and seeded; they are generated on the GPU before timing.

One step = the whole hot path on that input: stencil assembly from the map Jacobians,
hierarchy setup (operator-induced interpolation, Galerkin levels, coarsest factor), and the
solve.  value = interior DoF x steps / wall time of the float64 steps; the float32-refined steps
are timed the same way beside them.  roofline = the dominant float64 level-0 kernel (HIP events
on the library's stream).  cpu_baseline = one whole step of the same workload by the float64
oracle on one host thread, run in a subprocess during the GPU legs; its solution gives both GPU
results' error against the float64 oracle.

Extra legs (same JSON line): the same pair at 1025 x 1025, the batch of 256 uneven instances,
the differentiable solve on 2049 x 2049 with its finite-difference check, the grid <-> mesh
transfers, the two-level cycle on star meshes (and the paper's own configuration of it), the
quarter annulus with point and line smoothing, the discontinuous-coefficient problems.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--n 4097] [--no-c2] [--no-c4] [--no-c5]
                    [--no-transfer] [--no-twolevel] [--no-annulus] [--no-disc] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoF/s solved to 1e-10 rel. residual (FP64 vs FP32-refined) + % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(n: int, seed: int, device):
    import torch

    import problems as pb
    prob = pb.star(n, seed=seed, device="cuda" if device.type == "cuda" else None)
    as_dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()
    return prob, as_dev(prob.jac), as_dev(prob.K), as_dev(prob.b)


def run_leg(dmg, jac, K, b, steps: int, warmup: int, precision: int, inner: int = 1):
    """Times `steps` whole steps (assemble + refresh + solve) after `warmup` untimed ones."""
    import torch
    n_y, n_x = b.shape
    S = torch.empty((5, n_y, n_x), dtype=torch.float64, device=b.device)
    dmg.assemble_stencil(jac, K, out=S)
    h = dmg.Hierarchy(S, precision=precision, inner_cycles=inner)
    # launch shapes (rounding-level effect only) and, for float32 refinement, the float32 cycles per
    # refinement step (fastest solve to the same tolerance)
    info = {"tuned": h.autotune(b, tiles=True, reps=5, inner_cycles=precision == dmg.DMG_FP32_IR)}
    u = torch.zeros_like(b)

    def step():
        # the fine stencil assembled straight into the hierarchy, then its coarse levels
        h.refresh_assembled(jac, K)
        u.zero_()
        _, k, rel, _ = h.solve(b, u=u, rtol=1e-10)
        info["iters"], info["relres"] = k, rel

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info["wall_s"] = wall
    info["gpu_ms"] = ev0.elapsed_time(ev1)
    # solve-only rate on the prepared hierarchy (same u, b, stream: graph replay)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        h.solve(b, u=u, rtol=1e-10)
    torch.cuda.synchronize()
    info["solve_wall_s"] = time.perf_counter() - t0
    return h, u, info


def level0_kernel(h, n_x: int, n_y: int, kind: int):
    """Name and launch shape of the level-0 sweep kernel the hierarchy runs (kind 0 pre with
    restriction, 1 prolongation with post), as rocprofv3 lists it."""
    bw, seg_h = h.config()["levels" if kind == 0 else "post_levels"][0]
    wave = bw == 1
    width = 64 if wave else bw
    out_w = width - 12
    tiles = -(-n_x // out_w) * -(-n_y // seg_h)
    blocks = (tiles + 7) // 8 * 8
    mode = 1 if kind == 0 else 2
    name = f"k_wave<double, {mode}" if wave else f"k_strip<double, {bw}, {mode}"
    return dict(name=name, grid=blocks * width, workgroup=width, seg_h=seg_h)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2509_08109_amd", "csrc", "fused_kernels.hip")


def measured_traffic(kernel: dict, workload: str):
    """HBM bytes per launch of this kernel from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when none matches this kernel, launch shape and kernel source."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(KERNEL_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    for line in open(TRAFFIC_FILE):
        if not line.startswith("kernel="):
            continue
        kv = dict(tok.split("=", 1) for tok in line.strip().split(" | "))
        if (kv["kernel"] == kernel["name"] and kv["workload"] == workload
                and int(kv["grid"]) == kernel["grid"] and kv["source_sha256"] == sha):
            return float(kv["traffic_bytes"])
    return None


def kernel_roofline(dmg, h, b, workload: str, reps: int = 20):
    """Average duration of the level-0 fused pre and post kernels (HIP events on the stream the
    library launches on) and their algorithmic HBM bytes."""
    import torch
    n_y, n_x = b.shape
    nc = ((n_x + 1) // 2) * ((n_y + 1) // 2)
    # algorithmic bytes per launch: read S(5) u b, P(8 per coarse point), e or write b_H
    # (1 per coarse point); write u.  = 8 (8 N + 9 N_c)
    bytes_per_launch = 8.0 * (8 * n_x * n_y + 9 * nc)
    u = torch.zeros_like(b)
    out = {}
    for kind, name in ((0, "pre"), (1, "post")):
        for _ in range(3):
            h.sweep(0, kind, u, b)
        # `reps` launches captured in one graph (as the solve runs them), replayed `replays`
        # times between two events on the launching stream: the gaps between kernels are the
        # graph's, not the host's submission
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                h.sweep(0, kind, u, b)
        g.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        replays = 3
        e0.record()
        for _ in range(replays):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        del g
        ms = e0.elapsed_time(e1) / (reps * replays)
        out[name] = dict(level0_kernel(h, n_x, n_y, kind), avg_us=round(1e3 * ms, 2),
                         gbs=round(bytes_per_launch / (ms * 1e-3) / 1e9, 1))
    dom = out[max(out, key=lambda k: out[k]["avg_us"])]
    achieved = dom["gbs"]
    traffic = measured_traffic(dom, workload)
    return dict(bound="hbm", kernel=f"{dom['name']}, *> level 0 (grid {dom['grid']})", achieved=achieved,
                peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                bytes_per_launch=bytes_per_launch, avg_us=dom["avg_us"], kernels=out)


def run_batch_leg(dmg, dev, steps: int, count: int = 256):
    """The batch workload: ``count`` independent star instances, sizes uniform over
    {129, 257, 513, 1025}^2, each with its own map deformation, K and b (root seed 3), solved to
    1e-10 together by the batched schedule.  Generation + assembly and setup are timed apart
    from the solves (solve-only rate = interior DoF of all instances x steps / wall)."""
    import torch

    from problems.batch_device import star_batch_device
    t0 = time.perf_counter()
    Ss, bs, sizes = [], [], []
    for n, jac, K, b in star_batch_device(count, device=dev):
        Ss.append(dmg.assemble_stencil(jac, K))
        bs.append(b)
        sizes.append(n)
        del jac, K
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    bt = dmg.BatchSolver(Ss)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tuned = bt.autotune(bs, reps=2, tiles=True, colour_order=True)
    us = [torch.zeros_like(b) for b in bs]
    _, its, rels = bt.solve(bs, us=us, rtol=1e-10)          # warm-up (schedule, graph capture)
    wall = 0.0
    for _ in range(steps):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, rels = bt.solve(bs, us=us, rtol=1e-10)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
    dof = sum((n - 2) ** 2 for n in sizes)
    bt.close()
    del Ss, bs, us
    torch.cuda.empty_cache()
    return {"value": round(dof * steps / wall, 1), "unit": "DoF/s", "instances": count,
            "dof": dof, "sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))},
            "cycles_min": min(its), "cycles_max": max(its), "max_relres": max(rels),
            "tuned_colour_orders": {str(n): list(map(list, o)) for n, o in
                                    sorted({n: o for n, o in zip(sizes, tuned["orders"])}.items())},
            "ms_per_batch_solve": round(1e3 * wall / steps, 2), "steps": steps,
            "generate_and_assemble_s": round(t_gen, 2), "setup_s": round(t_setup, 2)}


def run_diff_leg(dmg, dev, steps: int, n: int = 2049, n_dirs: int = 64):
    """Differentiable solve on the n x n star (root seed 4): J(u) = 1/2 ||u - u_t||^2 over the
    interior, forward (assemble + setup + solve) and backward (hierarchy recomputed, adjoint
    solve, dJ/dK per cell, dJ/db) timed; then central differences along n_dirs seeded random
    directions (dK = K z, db = z with z ~ N(0,1), eps = 1e-4, solves to 1e-13) against the
    adjoint's directional derivatives."""
    import torch

    prob, jac, K0, b0 = make_inputs(n, 4, dev)
    t = torch.as_tensor(prob.target, dtype=torch.float64, device=dev)
    del prob

    relres_tight = []

    def J_of(Kv, bv, rtol):
        # the finite-difference solves run to 1e-13 or until the residual stops falling
        u = dmg.DiffSolve.apply(Kv, bv, jac, rtol, 200, None, rtol >= 1e-10)
        if rtol < 1e-10:
            relres_tight.append(dmg.DiffSolve.last["forward"][1])
        d = (u - t)[1:-1, 1:-1]
        return 0.5 * (d * d).sum()

    K = K0.clone().requires_grad_(True)
    b = b0.clone().requires_grad_(True)
    for _ in range(2):                                   # warm-up (graph captures)
        J_of(K, b, 1e-10).backward()
    K.grad = None
    b.grad = None
    fwd = bwd = 0.0
    for _ in range(steps):
        K.grad = None
        b.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = J_of(K, b, 1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        fwd += t1 - t0
        bwd += time.perf_counter() - t1
    # finite differences against the adjoint gradient of a tight solve
    K.grad = None
    b.grad = None
    J_of(K, b, 1e-13).backward()
    gK, gb = K.grad.detach(), b.grad.detach()
    gen = torch.Generator(device=dev)
    gen.manual_seed(4)
    eps = 1e-4
    fd, ad = [], []
    with torch.no_grad():
        for _ in range(n_dirs):
            zK = torch.randn(K0.shape, generator=gen, device=dev, dtype=torch.float64) * K0
            zb = torch.randn(b0.shape, generator=gen, device=dev, dtype=torch.float64)
            zb[0, :] = 0.0
            zb[-1, :] = 0.0
            zb[:, 0] = 0.0
            zb[:, -1] = 0.0
            fK = (J_of(K0 + eps * zK, b0, 1e-13) - J_of(K0 - eps * zK, b0, 1e-13)) / (2 * eps)
            fb = (J_of(K0, b0 + eps * zb, 1e-13) - J_of(K0, b0 - eps * zb, 1e-13)) / (2 * eps)
            fd.append(torch.stack([fK, fb]))
            ad.append(torch.stack([(gK * zK).sum(), (gb * zb).sum()]))
    fd = torch.stack(fd)
    ad = torch.stack(ad)
    err = (torch.linalg.norm(fd - ad, dim=0) / torch.linalg.norm(ad, dim=0)).tolist()
    dof = (n - 2) ** 2
    del jac, K0, b0, K, b, gK, gb, t
    torch.cuda.empty_cache()
    return {"value": round(dof * steps / (fwd + bwd), 1), "unit": "DoF/s (forward + backward)",
            "grid": [n, n], "dof": dof, "forward_ms": round(1e3 * fwd / steps, 2),
            "backward_ms": round(1e3 * bwd / steps, 2), "steps": steps,
            "fd_directions": n_dirs, "fd_relerr_dK": err[0], "fd_relerr_db": err[1],
            "fd_solves_max_relres": max(relres_tight) if relres_tight else None}


def run_transfer_leg(dmg, dev, n: int = 1025, seed: int = 1, reps: int = 20):
    """Grid <-> mesh transfers on the n x n grid of the star (root seed `seed`): a jittered P1
    lattice with about n^2 / 0.28 vertices mapped through the same star map, the rasterised
    coupled mass (nq = 4).  Two forms: C and C^T assembled at creation (CSR products per apply),
    and matrix-free (the overlap sets stored, the integrals recomputed per apply).
    from_grid = CG2(M_p, C u_c) and to_grid = C^T CG2(M_p, r_p) are timed with HIP events (mean
    of `reps` back-to-back applies); the device bytes that hold C are reported for both."""
    import numpy as np
    import torch

    import problems as pb
    mp = pb.Star.random(pb.streams(seed)[0])
    m = pb.mesh_points_for_grid(n)
    t0 = time.perf_counter()
    mesh = pb.lattice_mesh(mp, m, np.random.default_rng(seed))
    t_mesh = time.perf_counter() - t0
    uc = torch.zeros((n, n), dtype=torch.float64, device=dev)
    uc[1:-1, 1:-1] = 1.0
    rp = torch.ones(mesh.nv, dtype=torch.float64, device=dev)
    up = torch.empty(mesh.nv, dtype=torch.float64, device=dev)
    rc = torch.empty((n, n), dtype=torch.float64, device=dev)

    def timed(T):
        out = {}
        for name, fn in (("from_grid", lambda: T.from_grid(uc, out=up)),
                         ("to_grid", lambda: T.to_grid(rp, out=rc))):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            torch.cuda._sleep(20_000_000)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            out[name + "_us"] = round(1e3 * e0.elapsed_time(e1) / reps, 1)
        return out

    t0 = time.perf_counter()
    T = dmg.Transfer(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=4, device=dev)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    nnzC, nnzM = T.nnz()
    c_bytes = T.memory()[0]
    out = timed(T)
    T.close()
    # algorithmic bytes of one apply: C (or C^T) once and M_p twice at 12 B per nonzero (value +
    # column index) plus 4 B row pointers, the CG2 vectors (r0 written; r0, q0 for q0 = M r0;
    # r1 from r0, q0; r0, r1 for p1; r0, r1 and the result for x2: 11 passes of nv float64 plus
    # the int32 permutation) and the grid vector (read or written once)
    bytes_apply = (12.0 * (nnzC + 2 * nnzM) + 4.0 * 3 * mesh.nv + 8.0 * 11 * mesh.nv + 4.0 * mesh.nv
                   + 8.0 * n * n)
    t0 = time.perf_counter()
    Tf = dmg.Transfer(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=4, device=dev,
                      matrix_free=True)
    torch.cuda.synchronize()
    t_create_mf = time.perf_counter() - t0
    mf_bytes, pairs = Tf.memory()
    mf = timed(Tf)
    Tf.close()
    return {"grid": [n, n], "mesh_vertices": int(mesh.nv), "mesh_triangles": int(mesh.tris.shape[0]),
            "nnz_C": nnzC, "nnz_M": nnzM, "mesh_s": round(t_mesh, 2), "create_s": round(t_create, 2),
            **out, "apply_bytes": bytes_apply,
            "from_grid_gbs": round(bytes_apply / (out["from_grid_us"] * 1e-6) / 1e9, 1),
            "to_grid_gbs": round(bytes_apply / (out["to_grid_us"] * 1e-6) / 1e9, 1),
            "C_device_bytes": c_bytes,
            "matrix_free": {"create_s": round(t_create_mf, 2), "overlap_pairs": pairs,
                            "C_device_bytes": mf_bytes, **mf}}


def run_twolevel_leg(dmg, dev, sizes=(129, 257, 513), seed: int = 1, reps: int = 3):
    """The two-level cycle on the physical P1 system of star meshes of growing size (grid n x n,
    mesh about n^2 / 0.28 vertices, log-normal K per triangle, f ~ U(-1, 1); lumped mass, exact
    coupled mass): cycles to 1e-10 of the initial residual, wall time per solve
    (mean of `reps` solves after one that captures the graph) and per cycle, one grid V-cycle
    timed alone with HIP events for the grid's share of a cycle, and Sec. 2.4's coarse-grid
    scaling: its 12-step Lanczos estimate (time) and the cycles of a solve that applies it; the
    same solve over the matrix-free coupled mass; and the paper's own configuration (CG2, nq = 4)."""
    import numpy as np
    import torch

    from problems.batch_device import star_dmg_device
    rows = []
    for n in sizes:
        t0 = time.perf_counter()
        jac, K, mesh, K_t, f = star_dmg_device(n, seed, dev)
        t_gen = time.perf_counter() - t0
        H = dmg.Hierarchy(dmg.assemble_stencil(jac, K))
        t0 = time.perf_counter()
        tl = dmg.TwoLevel(H, mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, K_t=K_t, nq=0, mass="lumped")
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t0
        ncol, nnz_A, _ = tl.info()
        fd = torch.as_tensor(f, dtype=torch.float64, device=dev)
        tl.solve(fd, rtol=1e-10)
        walls = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, k, rel, hist = tl.solve(fd, rtol=1e-10)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        wall = sum(walls) / len(walls)
        ec = torch.zeros((n, n), dtype=torch.float64, device=dev)
        rc = torch.zeros_like(ec)
        rc[1:-1, 1:-1] = 1.0
        for _ in range(3):
            H.vcycle(ec, rc)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(20):
            H.vcycle(ec, rc)
        e1.record()
        torch.cuda.synchronize()
        # Sec. 2.4's coarse-grid scaling: the 12-step Lanczos estimate from a seeded start
        # vector, and the cycles of a solve that applies it
        v0 = torch.as_tensor(np.random.default_rng(seed).uniform(-1.0, 1.0, (n, n)),
                             dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gamma, _ = tl.estimate_scaling(v0, 12)
        t_gamma = time.perf_counter() - t0
        tl.set_scaling(gamma)
        _, k_g, rel_g, _ = tl.solve(fd, rtol=1e-10, raise_on_fail=False)
        tl.set_scaling(1.0)
        # the paper's own configuration on the same mesh: two CG iterations on M_p and the
        # rasterised coupled mass (4 x 4 Gauss points per grid cell)
        tlp = dmg.TwoLevel(H, mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, K_t=K_t, nq=4, mass="cg2")
        try:
            _, k_p, rel_p, hist_p = tlp.solve(fd, rtol=1e-10, max_iters=100, raise_on_fail=False)
            paper = {"cycles": k_p, "relres": rel_p, "converged": bool(rel_p <= 1e-10),
                     "rate_last_5": round((hist_p[-1] / hist_p[-6]) ** 0.2, 4) if len(hist_p) > 5 else None}
        except dmg.DmgError as e:          # non-finite residual: the cycle diverged
            paper = {"cycles": None, "relres": None, "converged": False, "diverged": str(e)}
        tlp.close()
        # the same cycle over the matrix-free coupled mass (no C stored)
        tlm = dmg.TwoLevel(H, mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, K_t=K_t, nq=0, mass="lumped",
                           matrix_free=True)
        tlm.solve(fd, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, k_m, rel_m, _ = tlm.solve(fd, rtol=1e-10)
        torch.cuda.synchronize()
        matrix_free = {"cycles": k_m, "relres": rel_m, "solve_ms": round(1e3 * (time.perf_counter() - t0), 3)}
        tlm.close()
        free = int(mesh.dof.sum())
        rows.append({"grid": n, "mesh_vertices": int(mesh.nv), "unknowns": free,
                     "triangles": int(mesh.tris.shape[0]), "colours": ncol, "nnz_A": nnz_A,
                     "cycles": k, "relres": rel, "rate": round(rel ** (1.0 / k), 4),
                     "solve_ms": round(1e3 * wall, 3), "ms_per_cycle": round(1e3 * wall / k, 4),
                     "grid_vcycle_ms": round(e0.elapsed_time(e1) / 20, 4),
                     "unknowns_per_s": round(free / wall, 1),
                     "gen_s": round(t_gen, 2), "create_s": round(t_create, 2),
                     "scaling": {"gamma": round(gamma, 4), "estimate_s": round(t_gamma, 3),
                                 "cycles_with_gamma": k_g, "relres_with_gamma": rel_g},
                     "paper_configuration_cg2_nq4": paper, "matrix_free_C": matrix_free})
        log(f"two-level {n}: {k} cycles, {1e3 * wall:.2f} ms, create {t_create:.1f} s; "
            f"matrix-free C {k_m} cycles {matrix_free['solve_ms']} ms; paper configuration (CG2, nq = 4): {paper}")
        tl.close()
        H.close()
    return {"workload": "star meshes, physical P1 system, lumped mass, exact coupled mass, FP64 grid V(1,1), "
                        "rtol 1e-10 relative to the initial residual", "sizes": rows}


def run_discontinuous_leg(dmg, dev, n: int = 513):
    """The paper's variable-coefficient problems on the unit square (identity map; diffusivity
    100 in a disc of radius 3/5, on a 4 x 4 checkerboard, or 1e-10 in a stripe of width 0.06;
    K per cell = mean at the Gauss points, K per triangle at the centroid): grid solves and
    two-level solves (lumped mass, exact C) to 1e-10, cycles and wall time; a two-level solve that
    does not converge in 300 cycles is reported as such."""
    import numpy as np
    import torch

    import problems as pb
    out = {}
    for kind in pb.DISCONTINUOUS:
        D = pb.discontinuous_dmg(kind, n)
        P = D.grid
        as_dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
        H = dmg.Hierarchy(dmg.assemble_stencil(as_dev(P.jac), as_dev(P.K)))
        b = as_dev(P.b)
        H.solve(b, rtol=1e-10, max_iters=300, raise_on_fail=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, k_g, rel_g, _ = H.solve(b, rtol=1e-10, max_iters=300, raise_on_fail=False)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t0
        m = D.mesh
        tl = dmg.TwoLevel(H, m.xy_c, m.xy_p, m.tris, m.dof, K_t=D.K_t)
        f = as_dev(D.f)
        try:
            tl.solve(f, rtol=1e-10, max_iters=300, raise_on_fail=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, k_t, rel_t, _ = tl.solve(f, rtol=1e-10, max_iters=300, raise_on_fail=False)
            torch.cuda.synchronize()
            t_t = time.perf_counter() - t0
        except dmg.DmgError as e:      # the iterates overflowed: the cycle diverges here
            k_t, rel_t, t_t = None, float("inf"), float("nan")
            log(f"{kind}: two-level solve diverged ({e})")
        out[kind] = {"grid_cycles": k_g, "grid_relres": rel_g, "grid_solve_ms": round(1e3 * t_g, 3),
                     "mesh_vertices": int(m.nv), "twolevel_cycles": k_t, "twolevel_relres": rel_t,
                     "twolevel_converged": bool(rel_t <= 1e-10),
                     "twolevel_solve_ms": round(1e3 * t_t, 3)}
        log(f"{kind}: grid {k_g} cycles, two-level {k_t} cycles (rel. residual {rel_t:.1e})")
        if not np.isfinite(out[kind]["twolevel_solve_ms"]):
            out[kind]["twolevel_solve_ms"] = None
        if not np.isfinite(rel_t):
            out[kind]["twolevel_relres"] = None
        tl.close()
        H.close()
    return {"grid": [n, n], "workload": "unit square, identity map, discontinuous diffusivity", **out}


def run_annulus_leg(dmg, dev, sizes=(65, 1025), reps: int = 5):
    """The quarter annulus (the paper's quarter annulus map, K = 1, b ~ U(-1, 1)): its pull-back
    is anisotropic (coupling along x up to 10x that along y), so 4-colour point smoothing
    converges slowly; the same solve with alternating zebra line relaxation, in float64 and as
    float32 line-smoothed cycles inside float64 refinement (one float32 cycle per step).  Cycles
    (refinement: outer steps) and solve wall time (mean of `reps` solves after one that captures
    the graph)."""
    import numpy as np
    import torch

    import problems as pb
    rows = []
    for n in sizes:
        prob = pb.quarter_annulus(n)
        as_dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
        S = dmg.assemble_stencil(as_dev(prob.jac), as_dev(prob.K))
        b = as_dev(prob.b)
        row = {"grid": n}
        for name, sm, prec in (("point", 0, dmg.DMG_FP64), ("alternating_lines", 3, dmg.DMG_FP64),
                               ("alternating_lines_fp32_refined", 3, dmg.DMG_FP32_IR)):
            h = dmg.Hierarchy(S, smoother=sm, precision=prec)
            h.solve(b, rtol=1e-10, max_iters=300, raise_on_fail=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                _, k, rel, _ = h.solve(b, rtol=1e-10, max_iters=300, raise_on_fail=False)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            row[name] = {"cycles": k, "relres": rel, "solve_ms": round(1e3 * wall, 3),
                         "dof_per_s": round((n - 2) ** 2 / wall, 1)}
            h.close()
        log(f"annulus {n}: point {row['point']['cycles']} cycles {row['point']['solve_ms']} ms, "
            f"lines {row['alternating_lines']['cycles']} cycles {row['alternating_lines']['solve_ms']} ms, "
            f"lines in float32 refinement {row['alternating_lines_fp32_refined']['cycles']} steps "
            f"{row['alternating_lines_fp32_refined']['solve_ms']} ms")
        rows.append(row)
    return {"workload": "quarter annulus, K = 1, V(1,1) to 1e-10 (FP64, and FP32 cycles in FP64 "
                        "refinement)", "sizes": rows}


CPU_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
from oracle import boxmg, cycle, fem
for job in {jobs!r}:
    d = np.load(job["inputs"])
    jac, K, b = d["jac"], d["K"], d["b"]
    ny, nx = b.shape
    t0 = time.perf_counter()
    S = fem.assemble_stencil(jac, K, nx, ny)
    t1 = time.perf_counter()
    orc = cycle.Oracle(boxmg.build_hierarchy(S))
    t2 = time.perf_counter()
    u, k, hist, _ = cycle.solve(orc, b, 1e-10)
    t3 = time.perf_counter()
    np.save(job["out"], u)
    print(json.dumps(dict(n=nx, assemble_s=t1 - t0, setup_s=t2 - t1, solve_s=t3 - t2, seconds=t3 - t0,
                          iters=k, relres=hist[-1], dof=(nx - 2) * (ny - 2))), flush=True)
    del d, jac, K, b, S, orc, u
"""


class OracleBaseline:
    """The float64 oracle on the host, one thread, one whole step (assemble + setup + solve to
    1e-10) of each given workload, run in a subprocess that starts before the GPU legs so that its
    CPU time overlaps them.  Its inputs are the arrays the GPU legs use (written to a temporary
    directory); its solutions come back so that every GPU result can state its error against the
    float64 oracle."""

    def __init__(self, workloads):
        import tempfile

        import numpy as np
        self.dir = tempfile.mkdtemp(prefix="dmg_oracle_")
        jobs = []
        for name, jac, K, b in workloads:
            path = os.path.join(self.dir, f"{name}_inputs.npz")
            np.savez(path, jac=jac, K=K, b=b)
            jobs.append(dict(name=name, inputs=path, out=os.path.join(self.dir, f"{name}_u.npy")))
        self.jobs = jobs
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
            env[k] = "1"
        env["CUDA_VISIBLE_DEVICES"] = ""
        env["HIP_VISIBLE_DEVICES"] = ""
        self.t0 = time.perf_counter()
        self.proc = subprocess.Popen([sys.executable, "-c", CPU_SNIPPET.format(root=ROOT, jobs=jobs)],
                                     stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)

    def results(self, timeout: float = 900.0):
        """{name: (stats dict, solution [ny][nx])} once the subprocess has finished."""
        import shutil

        import numpy as np
        out, err = self.proc.communicate(timeout=timeout)
        if self.proc.returncode != 0:
            raise RuntimeError(err[-2000:])
        stats = [json.loads(line) for line in out.strip().splitlines() if line.startswith("{")]
        res = {job["name"]: (st, np.load(job["out"])) for job, st in zip(self.jobs, stats)}
        shutil.rmtree(self.dir, ignore_errors=True)
        return res


def oracle_error(x, u_or):
    """||x - u_or|| / ||u_or|| and max |x - u_or| / max |u_or| of a GPU solution x (tensor)."""
    import numpy as np
    xh = x.detach().cpu().numpy()
    d = xh - u_or
    return {"rel_l2": float(np.linalg.norm(d) / np.linalg.norm(u_or)),
            "max_abs_over_max": float(np.abs(d).max() / np.abs(u_or).max())}


def device_inputs(n: int, seed: int, dev):
    """The star workload's map Jacobians at the Gauss points, log-normal K and b, generated on the
    device from the seeded streams of ``problems.star(n, seed)``."""
    from problems.batch_device import star_device
    return star_device(n, seed, dev)


def precision_legs(dmg, jac, K, b, steps: int, warmup: int, workload: str):
    """float64 and float32-refined legs of one workload: whole steps timed, solve-only rates, the
    roofline of the dominant float64 level-0 kernel."""
    n_y, n_x = b.shape
    dof = (n_x - 2) * (n_y - 2)
    h, u, i64 = run_leg(dmg, jac, K, b, steps, warmup, dmg.DMG_FP64)
    levels, gc, oc = h.stats()
    log(f"{workload} fp64: {i64['iters']} cycles, {1e3 * i64['wall_s'] / steps:.2f} ms/step")
    roof = kernel_roofline(dmg, h, b, workload)
    log(f"{workload} roofline: {roof['kernel']} {roof['avg_us']} us, {roof['achieved']} GB/s")
    u64 = u.clone()
    h.close()
    h32, x32, i32 = run_leg(dmg, jac, K, b, steps, warmup, dmg.DMG_FP32_IR)
    log(f"{workload} fp32-refined: {i32['iters']} steps of {i32['tuned']['inner_cycles']} float32 cycles, "
        f"{1e3 * i32['wall_s'] / steps:.2f} ms/step")
    x32 = x32.clone()
    h32.close()
    fp64 = {"value": round(dof * steps / i64["wall_s"], 1), "unit": "DoF/s",
            "ms_per_step": round(1e3 * i64["wall_s"] / steps, 3),
            "solve_only_dof_per_s": round(dof * steps / i64["solve_wall_s"], 1),
            "iters": i64["iters"], "relres": i64["relres"]}
    fp32 = {"value": round(dof * steps / i32["wall_s"], 1), "unit": "DoF/s",
            "ms_per_step": round(1e3 * i32["wall_s"] / steps, 3),
            "solve_only_dof_per_s": round(dof * steps / i32["solve_wall_s"], 1),
            "outer_steps": i32["iters"], "inner_cycles": i32["tuned"]["inner_cycles"],
            "relres": i32["relres"],
            "speedup_vs_fp64": round(i64["wall_s"] / i32["wall_s"], 3),
            "solve_only_speedup_vs_fp64": round(i64["solve_wall_s"] / i32["solve_wall_s"], 3)}
    info = {"levels": levels, "grid_complexity": round(gc, 4), "operator_complexity": round(oc, 4)}
    return fp64, fp32, roof, info, u64, x32


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4097, help="grid of the headline workload")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-c2", action="store_true", help="skip the 1025 x 1025 legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-c4", action="store_true", help="skip the 256-instance batch leg")
    ap.add_argument("--no-c5", action="store_true", help="skip the 2049 x 2049 gradient leg")
    ap.add_argument("--no-transfer", action="store_true", help="skip the grid <-> mesh transfer leg")
    ap.add_argument("--no-twolevel", action="store_true", help="skip the two-level mesh cycle leg")
    ap.add_argument("--no-disc", action="store_true", help="skip the discontinuous-coefficient leg")
    ap.add_argument("--no-annulus", action="store_true", help="skip the quarter-annulus smoother leg")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_08109_amd as dmg
    dmg.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)   # graph capture needs a non-default stream

    # a plain streaming kernel of known size (an elementwise multiply by one: 512 MiB read,
    # 512 MiB written); the HBM byte counters of the sweep kernels are scaled by what the same
    # counters report for it
    calib = torch.ones(64 << 20, dtype=torch.float64, device=dev)
    calib_dst = torch.empty_like(calib)
    torch.mul(calib, 1.0, out=calib_dst)
    torch.cuda.synchronize()
    # its rate, reported beside the roofline as context: what a plain streaming kernel sustains
    # on this GPU (the roofline's peak stays the published figure)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        torch.mul(calib, 1.0, out=calib_dst)
    ev0.record(stream)
    for _ in range(20):
        torch.mul(calib, 1.0, out=calib_dst)
    ev1.record(stream)
    torch.cuda.synchronize()
    stream_gbs = 2 * calib.numel() * 8 * 20 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del calib, calib_dst

    n, n2 = args.n, 1025
    log(f"generating the {n}x{n} star workload (root seed {args.seed}) on the device")
    jac, K, b = device_inputs(n, args.seed, dev)
    c2 = None if args.no_c2 else device_inputs(n2, 1, dev)
    oracle = None
    if not args.no_cpu:
        host = lambda t: t.detach().cpu().numpy()
        work = [("headline", host(jac), host(K), host(b))]
        if c2 is not None:
            work.append(("c2", *(host(t) for t in c2)))
        oracle = OracleBaseline(work)
        del work
        log("oracle baseline started (one thread, in the background)")
    dof = (n - 2) ** 2
    workload = f"{n}x{n}"
    fp64, fp32, roof, info, u64, x32 = precision_legs(dmg, jac, K, b, args.steps, args.warmup, workload)
    del jac, K
    torch.cuda.empty_cache()
    res = {
        "metric": METRIC, "value": fp64["value"], "unit": "DoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded star-domain map Jacobians, log-normal K, uniform RHS)",
        "config": {"workload": f"{n}x{n} star domain (root seed {args.seed}), log-normal K, "
                               "FP64 V(1,1) and FP32-refined solves to 1e-10 rel. residual; "
                               "step = assemble + setup + solve; value = FP64",
                   "grid": [n, n], "dof": dof, **info, "seed": args.seed},
        "iters": fp64["iters"], "relres": fp64["relres"],
        "solve_only_dof_per_s": fp64["solve_only_dof_per_s"],
        "fp64": fp64,
        "fp32_refined": fp32,
        "roofline": roof,
        "stream_reference": {"kernel": "torch.mul, float64, 512 MiB read + 512 MiB written",
                             "gbs": round(stream_gbs, 1), "frac_of_peak": round(stream_gbs / HBM_PEAK_GBS, 4)},
    }
    solutions = {"headline": (u64, x32)}
    del b
    if c2 is not None:
        jac2, K2, b2 = c2
        fp64_2, fp32_2, roof2, info2, u64_2, x32_2 = precision_legs(dmg, jac2, K2, b2, args.steps,
                                                                    args.warmup, f"{n2}x{n2}")
        res["c2_1025"] = {"workload": f"{n2}x{n2} star domain (root seed 1); fits in the 256 MB "
                                      "last-level cache, not an HBM roofline claim",
                          "fp64": fp64_2, "fp32_refined": fp32_2, "roofline": roof2, **info2}
        solutions["c2"] = (u64_2, x32_2)
        del jac2, K2, b2, c2
        torch.cuda.empty_cache()
    if not args.no_c4:
        log("batch leg: 256 star instances")
        res["c4_batch"] = run_batch_leg(dmg, dev, max(1, args.steps // 2))
    if not args.no_c5:
        log("gradient leg: 2049x2049 star")
        res["c5_gradient"] = run_diff_leg(dmg, dev, max(4, args.steps))
    if not args.no_transfer:
        log("transfer leg: 1025x1025 grid, ~3.8M-vertex mesh")
        res["transfer"] = run_transfer_leg(dmg, dev)
    if not args.no_twolevel:
        log("two-level leg: star meshes at grids 129, 257, 513")
        res["twolevel"] = run_twolevel_leg(dmg, dev)
    if not args.no_annulus:
        log("quarter-annulus leg: point vs line smoothing")
        res["annulus"] = run_annulus_leg(dmg, dev)
    if not args.no_disc:
        log("discontinuous-coefficient leg: 513x513 unit square")
        res["discontinuous"] = run_discontinuous_leg(dmg, dev)
    if oracle is not None:
        log("waiting for the oracle baseline")
        got = oracle.results()
        st, u_or = got["headline"]
        res["cpu_baseline"] = dict(
            value=st["dof"] / st["seconds"], unit="DoF/s", cores=1, kind="oracle",
            sample=f"one whole step (assemble + setup + solve to 1e-10, {st['iters']} V-cycles) of the "
                   f"{n}x{n} workload, float64 NumPy/SciPy, one thread",
            seconds=round(st["seconds"], 2), assemble_s=round(st["assemble_s"], 2),
            setup_s=round(st["setup_s"], 2), solve_s=round(st["solve_s"], 2),
            solve_only_dof_per_s=round(st["dof"] / st["solve_s"], 1), iters=st["iters"],
            host_cpus=os.cpu_count())
        res["fp64"]["error_vs_fp64_oracle"] = oracle_error(solutions["headline"][0], u_or)
        res["fp32_refined"]["error_vs_fp64_oracle"] = oracle_error(solutions["headline"][1], u_or)
        res["fp64"]["oracle_iters"] = st["iters"]
        if "c2" in got:
            st2, u_or2 = got["c2"]
            res["c2_1025"]["fp64"]["error_vs_fp64_oracle"] = oracle_error(solutions["c2"][0], u_or2)
            res["c2_1025"]["fp32_refined"]["error_vs_fp64_oracle"] = oracle_error(solutions["c2"][1], u_or2)
            res["c2_1025"]["cpu_oracle"] = dict(value=st2["dof"] / st2["seconds"], unit="DoF/s", cores=1,
                                                seconds=round(st2["seconds"], 2), iters=st2["iters"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
