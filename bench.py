#!/usr/bin/env python3
"""Benchmark of the whole hot path on one MI355X.

One step = one pass of the path over one batch of synthetic input: host mesh analysis and near
list, device assembly of W (far 7x7 tiles, Duffy near kernels, contraction, FP32 copy), right-hand
sides, preconditioner set-up (batched block inverses, coarse Galerkin matrix), and the
mixed-precision PCG solve of k right-hand sides to relative residual tol.  Every solved column is
checked against an FP64 reference solution (FP64 GPU PCG at relative residual 1e-13, computed
before the timed region); only columns with relative error <= 1e-8 count.

Prints one JSON line (see the "metric"/"value" keys); per-phase timings, matvec bandwidths, the
roofline of the dominant kernel and the oracle timed on the host cores ride along.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
# algorithmic FP64 flops of one far-field kernel evaluation w / |x - y| as the far kernel issues it
# (counted in its gfx950 ISA): 3 subtractions, 1 product and 2 FMAs for |x-y|^2, 2 products and 1
# FMA for the Newton step of the reciprocal square root, 1 FMA into the inner sum, and 1 FMA per
# 7 evaluations into the outer sum; an FMA counts 2, the v_rsq_f64 estimate is not counted
FLOPS_PER_EVAL = 14.0 + 2.0 / 7.0
EVALS_PER_FAR_PAIR = 49


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def far_kernel_source_hash():
    """Hash of the far-field pass's own source text (its constants and its three kernels, through
    the far kernel's closing brace), so that counters taken on an older version are not reported."""
    src = open(os.path.join(ROOT, "paper_2310_09204_amd", "csrc", "assemble.hip")).read()
    a = src.index("constexpr int kGrp")
    b = src.index("\n}\n", src.index("void k_far(", a)) + 3
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def symv_bytes(N, size):
    """HBM bytes of one symmetric product (any number of columns up to 16): the upper block triangle of W
    (64 x 64 blocks) plus the block-row partials written and read back (super-blocks of 8 blocks
    for FP32 and 4 for FP64 matrices; one partial of 64 rows x 16 columns per block row and
    super-tile, plus one)."""
    nb = (N + 63) // 64
    ks = 8 if size == 4 else 4
    nst = (nb + ks - 1) // ks
    return nb * (nb + 1) // 2 * 64 * 64 * size + 2 * nb * (nst + 1) * 1024 * size


def matvec_rates(N, size, t, key):
    """A product's time, its HBM rate and the full-matrix equivalent rate (N^2 entries / t)."""
    return {key + "_ms": t * 1e3, key + "_hbm_GBs": symv_bytes(N, size) / t / 1e9,
            key + "_equiv_GBs": N * N * size / t / 1e9}


def load_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if the kernel source is
    unchanged since the counters were taken; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(kernel, {}).get(workload)
        if not e or e.get("source_hash") != far_kernel_source_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(w, k, iters, gpu_info, budget_s):
    """The oracle on the host cores, on a bounded sample of this workload, scaled to solves/s.

    Sample: R random rows of the pair-integral matrix (all columns; far and near pairs exactly as
    the oracle assembles them) timed with oracle_I_rows; the dense products of the PCG timed on a
    slab of rows of a matrix of the workload's size; scaled to N_T rows and to the solve's
    iteration count.  The oracle's contraction and preconditioner set-up are not included (so
    the baseline is optimistic for the oracle)."""
    from oracle import native
    from oracle.assemble import _tables
    import ctypes

    V = np.ascontiguousarray(w.mesh.vertices, dtype=np.float64)
    T = np.ascontiguousarray(w.mesh.triangles, dtype=np.int32)
    nt = T.shape[0]
    N = int(gpu_info["n_dofs"])
    b7, w7, gx, gw = _tables(10)
    L = native.lib()
    rng = np.random.default_rng(0)
    # calibrate: one row first
    rows_done, t_rows = 0, 0.0
    R = 1
    buf = np.empty((64, nt))
    while t_rows < 0.6 * budget_s and rows_done < nt:
        R = min(R, 64)
        r0 = int(rng.integers(0, nt - R))
        t0 = time.perf_counter()
        L.oracle_I_rows(native.dptr(V), native.iptr(T), nt, native.dptr(b7), native.dptr(w7), 10,
                        native.dptr(gx), native.dptr(gw), r0, R, native.dptr(buf))
        t_rows += time.perf_counter() - t0
        rows_done += R
        R *= 2
    t_asm = t_rows / rows_done * nt
    # dense matvec slab: W[rows, :] @ X, k columns
    slab = 1024
    Wslab = rng.standard_normal((slab, N))
    X = rng.standard_normal((N, k))
    reps, t_mv = 0, 0.0
    while t_mv < 0.2 * budget_s and reps < 50:
        t0 = time.perf_counter()
        Wslab @ X
        t_mv += time.perf_counter() - t0
        reps += 1
    t_matvec = t_mv / reps * (N / slab)
    t_solve = iters * t_matvec
    t_step = t_asm + t_solve
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": k / t_step,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d of %d rows of the pair-integral matrix (oracle_I_rows, all columns) and a %d-row slab "
                  "of the dense %d-column product, scaled to one step of %d right-hand sides with %d PCG "
                  "iterations; contraction and preconditioner set-up not counted" % (rows_done, nt, slab, k, k, iters),
        "t_assembly_s": t_asm,
        "t_solve_s": t_solve,
        "pair_integrals_per_s": nt * (nt + 1) / 2 / t_asm,
    }


def _replay(lib, reqs, ctx, scale, max_inflight):
    """Submits reqs at t_arrival * scale (scale 0: all at once) and polls them in order."""
    import threading
    srv = lib.Server(ctx, max_inflight=max_inflight)
    tickets = [None] * len(reqs)
    t0 = time.perf_counter()

    def feeder():
        for i, r in enumerate(reqs):
            dt = r.t_arrival * scale - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(r.mesh.vertices, r.mesh.triangles, r.patch_of_triangle, r.coarse.vertices,
                                    r.coarse.triangles, r.coarse_of_triangle, r.g,
                                    precision=lib.FP32_REFINE if r.mixed else lib.FP64, tol=1e-10)

    th = threading.Thread(target=feeder)
    th.start()
    results = []
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(1e-4)
        results.append(srv.poll(tickets[i]) + (srv.last_message,))
    t_end = time.perf_counter()
    th.join()
    stats = srv.stats()
    srv.close()
    return results, t_end - t0, stats


def serving_leg(lib, meshes, ctx, n_requests, load, seed=0, max_inflight=4):
    """Seeded Poisson stream of solve requests on random multiscreens (N ~ U[2k, 30k], 1-16 g per
    request, FP64 or mixed), replayed in real time into the serving loop.

    Capacity is measured first by submitting the whole stream at once; the timed replay then
    scales the seeded arrival times to `load` x capacity.  Latency is submit -> completion as the
    server measures it; solves/s counts right-hand sides within rel.err 1e-8 of an FP64 solve of
    the same request (computed after the stream, not timed)."""
    reqs = meshes.serving_stream(seed, n_requests, rate=1.0)    # arrival times for rate 1/s
    res_b, t_burst, _ = _replay(lib, reqs, ctx, 0.0, max_inflight)
    for i, res in enumerate(res_b):
        if res[2] < 0:
            log("bench: serving request %d failed in the burst: rc %d %s" % (i, res[2], res[3]))
    capacity = n_requests / t_burst                              # requests/s
    rate = load * capacity
    results, t_run, stats = _replay(lib, reqs, ctx, 1.0 / rate, max_inflight)
    solved, worst = 0, 0.0
    by_geo = {}
    total = sum(r.g.shape[0] for r in reqs)
    failed = [(i, res[2], res[3]) for i, res in enumerate(results) if res[2] < 0]
    for i, rc, msg in failed:
        log("bench: serving request %d failed: rc %d %s" % (i, rc, msg))
    for r, res in zip(reqs, results):
        if res[2] >= 0:
            by_geo.setdefault(r.geometry, []).append((r, res[:3]))
    for items in by_geo.values():
        r0 = items[0][0]
        p = lib.Problem(ctx, r0.mesh.vertices, r0.mesh.triangles)
        M = lib.Preconditioner(p, r0.patch_of_triangle, r0.coarse.vertices, r0.coarse.triangles,
                               r0.coarse_of_triangle)
        for r, (phi, info, rc) in items:
            ref, _, _ = p.solve(g=r.g, precond=M, tol=1e-13)
            err = np.linalg.norm(phi - ref, axis=1) / np.linalg.norm(ref, axis=1)
            solved += int((err <= 1e-8).sum())
            worst = max(worst, float(err.max()))
        M.close()
        p.close()
    lat = sorted(res[1][0]["t_total_s"] for res in results)
    n_dofs = [int(res[0].shape[1]) for res in results]
    return {
        "requests": len(reqs), "failed_requests": len(failed),
        "direct_launch_requests": sum(1 for res in results if res[2] >= 0 and res[1][0]["graph"] == 0), "rhs": total, "rhs_within_1e-8": solved, "relerr_max": worst,
        "capacity_requests_per_s": capacity, "load": load, "arrival_rate_per_s": rate,
        "max_inflight": max_inflight,
        "solves_per_s": solved / t_run,
        "latency_s": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]},
        "n_dofs_range": [min(n_dofs), max(n_dofs)],
        "mixed_requests": int(sum(r.mixed for r in reqs)),
        "server": stats,
    }


def double_layer_leg(lib, w, ctx, m_targets=16384, k=16):
    """Double-layer potential (Lemma repDL) of k crossed96 solutions at seeded targets in [-1, 1]^3
    at least 0.05 (about 5 h) from every panel plane: evaluations (target x Gauss point) per second
    and the FP64 rate, counting 16 + 2 k flops per evaluation (distance 8, Newton step 4, cube 2,
    normal projection 2, one FMA per column; the reciprocal square root not counted)."""
    m = w.mesh
    p = lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE, near_order=10)
    M = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                           factor_fp32=True)
    g = w.g[:k] if w.g.shape[0] >= k else np.resize(w.g, (k, 3))
    phi, _, _ = p.solve(g=g, precond=M, tol=1e-10, precision=lib.FP32_REFINE)
    rng = np.random.default_rng(11)
    X = []
    while len(X) < m_targets:
        x = rng.uniform(-1.0, 1.0, size=(m_targets, 3))
        X.extend(x[np.abs(x).min(axis=1) >= 0.05])
    X = np.array(X[:m_targets])
    p.double_layer(phi, X)     # builds the per-triangle records
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        U = p.double_layer(phi, X)
    t = (time.perf_counter() - t0) / reps
    evals = m_targets * 7 * m.nt
    out = {"targets": m_targets, "k": k, "t_s": t, "evals_per_s": evals / t,
           "tflops": evals * (16 + 2 * k) / t / 1e12, "finite": bool(np.isfinite(U).all())}
    M.close()
    p.close()
    log("bench: double layer %d targets x %d points, k=%d: %.2f ms, %.1f TFLOP/s" %
        (m_targets, 7 * m.nt, k, t * 1e3, out["tflops"]))
    return out


def planar_leg(lib, meshes, ctx):
    """Section 2's planar experiments on the GPU path.  Experiment 1: the plus-shaped cross with
    g = (0, -1/2) on uniform and tip-graded meshes (grading 2, node k at 1 - (1 - k/n)^2 of an arm);
    discrete l2 error of U_h against the exact field on a 61 x 61 grid over [-1.5, 1.5]^2 (shifted off
    the arms), CG iterations and the time of assembly + solve.  Experiment 2: the threefold junction
    with faces = coarse segments; Lanczos estimates of kappa(P_ad W) and kappa(W) over H and H/h."""
    g = np.linspace(-1.5, 1.5, 61) + 0.0123
    X = np.array([(a, b) for a in g for b in g])
    exact = meshes.cross_solution(X)
    exp1 = []
    for grading in (1.0, 2.0):
        for n in (16, 32, 64, 128, 256, 512):
            V, S = meshes.plus2d(n, grading)
            t0 = time.perf_counter()
            p = lib.Problem2D(ctx, V, S)
            phi, info, rc = p.solve(g=np.array([0.0, -0.5]), precond=None, tol=1e-12)
            t1 = time.perf_counter()
            U = p.double_layer(phi, X)[0]
            exp1.append({"grading": grading, "segments_per_arm": n, "n_dofs": p.N, "cg_iters": info[0]["iters"],
                         "t_assemble_solve_s": t1 - t0, "l2_error": float(np.sqrt(np.mean((U - exact) ** 2)))})
            p.close()
    exp2 = []
    for nc in (2, 4, 8):
        for r in (2, 4, 8, 16, 32):
            if nc * r > 256:
                continue
            (V, S), (cV, cS), par = meshes.arms2d_coarse("threefold", nc * r, r)
            p = lib.Problem2D(ctx, V, S)
            M = lib.Preconditioner(p, par, cV, cS, par)
            b = np.random.default_rng(nc * 100 + r).standard_normal((1, p.N))
            _, info, _ = p.solve(rhs=b, precond=M, tol=1e-12)
            _, info_cg, _ = p.solve(rhs=b, precond=None, tol=1e-12)
            exp2.append({"coarse_segments_per_arm": nc, "H_over_h": r, "n_dofs": p.N,
                         "kappa_pad": info[0]["est_cond"], "kappa_W": info_cg[0]["est_cond"],
                         "pcg_iters": info[0]["iters"], "cg_iters": info_cg[0]["iters"]})
            M.close()
            p.close()
    for e in exp1:
        log("bench: planar cross grading %.0f n=%d N=%d error %.3e (%d CG iterations, %.1f ms)" %
            (e["grading"], e["segments_per_arm"], e["n_dofs"], e["l2_error"], e["cg_iters"], e["t_assemble_solve_s"] * 1e3))
    for e in exp2:
        log("bench: threefold junction nH=%d H/h=%d kappa(P W)=%.3f kappa(W)=%.1f" %
            (e["coarse_segments_per_arm"], e["H_over_h"], e["kappa_pad"], e["kappa_W"]))
    return {"experiment1_cross": exp1, "experiment2_threefold": exp2}


def kappa_study(lib, meshes, ctx):
    """Lanczos estimate of kappa(P_ad W) on the paper's three-dimensional experiment (two
    perpendicular equilateral triangles sharing a median) with faces = coarse triangles, over coarse
    sizes H = (1/2, 1/4, 1/8) x edge and H/h = 2..16, next to kappa(W) (unpreconditioned CG) and
    the iteration counts; a seeded generic right-hand side, PCG to 1e-12."""
    rows = []
    for nc in (2, 4, 8):
        for ratio in (2, 4, 8, 16):
            n = nc * ratio
            if n > 128:
                continue
            m = meshes.bowtie(n)
            cm, par = meshes.bowtie_coarse(n, ratio)
            p = lib.Problem(ctx, m.vertices, m.triangles, near_order=10)
            M = lib.Preconditioner(p, par, cm.vertices, cm.triangles, par)
            b = np.random.default_rng(n * 100 + ratio).standard_normal((1, p.N))
            _, info, _ = p.solve(rhs=b, precond=M, tol=1e-12)
            _, info_cg, _ = p.solve(rhs=b, precond=None, tol=1e-12)
            _, info_g, _ = p.solve(g=meshes.BOWTIE_G, precond=M, tol=1e-10)
            sz = M.sizes()
            rows.append({"coarse_n": nc, "H_over_h": ratio, "n": n, "n_dofs": p.N, "n_faces": sz["n_faces"],
                         "n_wb": sz["n_wb"], "n_coarse": sz["n_coarse"],
                         "kappa_pad": info[0]["est_cond"], "kappa_W": info_cg[0]["est_cond"],
                         "pcg_iters": info[0]["iters"], "cg_iters": info_cg[0]["iters"],
                         "pcg_iters_g_1e-10": info_g[0]["iters"]})
            M.close()
            p.close()
            log("bench: kappa study n=%d H/h=%d N=%d kappa(P W)=%.3f kappa(W)=%.1f" %
                (n, ratio, rows[-1]["n_dofs"], rows[-1]["kappa_pad"], rows[-1]["kappa_W"]))
    return rows


def large_leg(lib, meshes, ctx, k=16):
    """crossed192 (N = 110,017; W 48 GB FP32 + 97 GB FP64, the pair matrix built in panels): a
    warm-up step, then one timed step (assembly, set-up, mixed-precision solve of k right-hand
    sides to relative residual 1e-10), the FP64 PCG solve of the same system beside it, and an
    FP64 reference (tol 1e-13) for the errors."""
    w = meshes.workload("crossed192", seed=0, k=k)
    m = w.mesh
    ctx.release_cached()

    def one_step():
        t0 = time.perf_counter()
        p = lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE, near_order=10)
        t1 = time.perf_counter()
        M = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles,
                               w.coarse_of_triangle, factor_fp32=True)
        t2 = time.perf_counter()
        phi, info, rc = p.solve(g=w.g, precond=M, tol=1e-10, precision=lib.FP32_REFINE)
        t3 = time.perf_counter()
        return p, M, phi, info, (t0, t1, t2, t3)

    p, M, _, _, (t0, t1, t2, t3) = one_step()
    first = t3 - t0
    M.close()
    p.close()
    p, M, phi, info, (t0, t1, t2, t3) = one_step()
    pinfo = p.info
    t4 = time.perf_counter()
    phi64, info64, _ = p.solve(g=w.g, precond=M, tol=1e-10, precision=lib.FP64)
    t5 = time.perf_counter()
    ref, _, _ = p.solve(g=w.g, precond=M, tol=1e-13, precision=lib.FP64)
    err = np.linalg.norm(phi - ref, axis=1) / np.linalg.norm(ref, axis=1)
    err64 = np.linalg.norm(phi64 - ref, axis=1) / np.linalg.norm(ref, axis=1)
    # the diagonal wire basket (Remark "Approximate solvers") on the same matrix
    t6 = time.perf_counter()
    Md = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                            factor_fp32=True, wirebasket="diagonal")
    t7 = time.perf_counter()
    phid, infod, _ = p.solve(g=w.g, precond=Md, tol=1e-10, precision=lib.FP32_REFINE)
    t8 = time.perf_counter()
    errd = np.linalg.norm(phid - ref, axis=1) / np.linalg.norm(ref, axis=1)
    Md.close()
    N = pinfo["n_dofs"]
    t32 = p.bench_matvec(fp32=True, k=16, reps=3)
    t64 = p.bench_matvec(fp32=False, k=16, reps=3)
    nt = m.nt
    step = t3 - t0
    out = {
        "workload": "crossed192: " + w.description, "n_dofs": N, "n_tri": nt, "k": k,
        "pair_panels": pinfo["n_pair_panels"],
        "t_step_s": step, "t_first_step_s": first, "t_assemble_s": t1 - t0, "t_precond_s": t2 - t1,
        "t_solve_s": t3 - t2, "t_far_s": pinfo["t_far_s"], "t_near_s": pinfo["t_near_s"],
        "t_contract_s": pinfo["t_contract_s"], "t_host_s": pinfo["t_host_s"],
        "solves_per_s": int((err <= 1e-8).sum()) / step,
        "iters": [i["iters"] for i in info], "relerr_max": float(err.max()),
        "fp64_solve": {"t_solve_s": t5 - t4, "iters": [i["iters"] for i in info64], "relerr_max": float(err64.max())},
        "diagonal_wirebasket": {"t_precond_s": t7 - t6, "t_solve_s": t8 - t7, "iters": [i["iters"] for i in infod],
                                "relerr_max": float(errd.max()),
                                "solves_per_s": int((errd <= 1e-8).sum()) / ((t1 - t0) + (t7 - t6) + (t8 - t7))},
        "pair_integrals_per_s": nt * (nt + 1) / 2 / (t1 - t0),
        "matvec": {**matvec_rates(N, 4, t32, "fp32_k16"), **matvec_rates(N, 8, t64, "fp64_k16")},
        "patches": M.sizes(),
    }
    M.close()
    p.close()
    ctx.release_cached()
    log("bench: crossed192 step %.3fs (first %.3fs) asm %.3f precond %.3f solve %.3f iters %s relerr %.2e"
        % (step, first, t1 - t0, t2 - t1, t3 - t2, out["iters"][:4], out["relerr_max"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="crossed96")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests in the serving-stream leg (0 skips it)")
    ap.add_argument("--no-large", action="store_true", help="skip the crossed192 leg")
    ap.add_argument("--no-kappa", action="store_true", help="skip the condition-number study")
    ap.add_argument("--no-potential", action="store_true", help="skip the double-layer potential leg")
    ap.add_argument("--no-planar", action="store_true", help="skip the two-dimensional experiments")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="arrival rate of the serving leg as a fraction of its measured capacity")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device-to-device three times (the reference launch that scales "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported (the multi-GPU "
              "design is described, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device-to-device copy", "bytes_read": src.numel() * 8,
                          "bytes_written": dst.numel() * 8, "launches": 3}))
        return

    from paper_2310_09204_amd import lib, meshes

    w = meshes.workload(args.workload, seed=0, k=args.k)
    m = w.mesh
    mixed = args.precision == "mixed"
    prec = lib.FP32_REFINE if mixed else lib.FP64
    log("bench: workload %s nt=%d k=%d precision=%s" % (args.workload, m.nt, args.k, args.precision))
    ctx = lib.Context(0)

    # the timed steps take the mesh from device memory and leave the solutions there (inputs resident
    # in HBM); host copies of the mesh still feed the host-side analysis
    d_mesh = (lib.DeviceArray(np.asarray(m.vertices, dtype=np.float64)),
              lib.DeviceArray(np.asarray(m.triangles, dtype=np.int32)))

    def step(precision, want_phi=False, tol=args.tol, wirebasket="exact", device_out=None):
        t0 = time.perf_counter()
        p = lib.Problem(ctx, m.vertices, m.triangles, precision=precision, near_order=10,
                        device_mesh=(d_mesh[0].ptr, d_mesh[1].ptr) if device_out is not None else None)
        t1 = time.perf_counter()
        M = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                               factor_fp32=(precision == lib.FP32_REFINE), wirebasket=wirebasket)
        t2 = time.perf_counter()
        phi, info, rc = p.solve(g=w.g, precond=M, tol=tol, precision=precision,
                                device_out=device_out.ptr if device_out is not None else None)
        ctx.synchronize()
        t3 = time.perf_counter()
        pinfo = p.info
        out = {"t_step": t3 - t0, "t_assemble": t1 - t0, "t_precond": t2 - t1, "t_solve": t3 - t2,
               "t_far": pinfo["t_far_s"], "t_near": pinfo["t_near_s"], "t_contract": pinfo["t_contract_s"],
               "t_host": pinfo["t_host_s"],
               "iters": [i["iters"] for i in info], "outer": [i["outer_iters"] for i in info], "rc": rc,
               "info": pinfo, "precond_sizes": M.sizes()}
        if want_phi:
            out["phi"] = phi
            out["problem"], out["M"] = p, M
        else:
            M.close()
            p.close()
        return out

    # reference solution (not timed)
    log("bench: FP64 reference solve (tol 1e-13)")
    ref = step(lib.FP64, want_phi=True, tol=1e-13)
    phi_ref = ref["phi"]
    pinfo = ref["info"]
    N = pinfo["n_dofs"]
    pref = ref["problem"]
    t64_1 = pref.bench_matvec(fp32=False, k=1, reps=10)
    t64_16 = pref.bench_matvec(fp32=False, k=16, reps=5)
    ref["M"].close()
    pref.close()

    # one device buffer per timed step for its solutions, allocated before the timed region
    d_out = [lib.DeviceArray(shape=(w.g.shape[0], N)) for _ in range(max(args.steps, 1))]
    for i in range(args.warmup):
        log("bench: warmup %d" % i)
        step(prec, device_out=d_out[0])
    ctx.synchronize()
    res = []
    t_begin = time.perf_counter()
    for i in range(args.steps):
        r = step(prec, want_phi=True, device_out=d_out[i])
        r.pop("phi")
        r.pop("M").close()
        r.pop("problem").close()
        res.append(r)
    ctx.synchronize()
    elapsed = time.perf_counter() - t_begin
    # checks and side measurements, outside the timed region
    phis = [d.get() for d in d_out[:args.steps]]
    for d in d_out:
        d.close()
    for i, (r, phi) in enumerate(zip(res, phis)):
        err = np.linalg.norm(phi - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        r["relerr"] = err.tolist()
        r["solved"] = int((err <= 1e-8).sum())
        log("bench: step %d %.3fs asm %.3f (host %.3f far %.3f near %.4f contract %.3f) precond %.3f solve %.3f iters %s relerr max %.2e"
            % (i, r["t_step"], r["t_assemble"], r["t_host"], r["t_far"], r["t_near"], r["t_contract"], r["t_precond"], r["t_solve"],
               r["iters"][:4], max(r["relerr"])))
    t32_1 = t32_16 = None
    if mixed:
        pl = lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE, near_order=10)
        t32_1 = pl.bench_matvec(fp32=True, k=1, reps=10)
        t32_16 = pl.bench_matvec(fp32=True, k=16, reps=5)
        pl.close()
    solved = sum(r["solved"] for r in res)
    value = solved / elapsed
    ms_per_step = elapsed / args.steps * 1e3

    fp64_step = None
    if not args.no_fp64_compare and mixed:
        r64 = step(lib.FP64, want_phi=True)
        err64 = np.linalg.norm(r64["phi"] - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        r64["M"].close()
        r64["problem"].close()
        fp64_step = {"t_step_s": r64["t_step"], "t_solve_s": r64["t_solve"], "iters": r64["iters"],
                     "solves_per_s": int((err64 <= 1e-8).sum()) / r64["t_step"],
                     "solve_only_solves_per_s": int((err64 <= 1e-8).sum()) / r64["t_solve"]}

    # the same step with the diagonal wire basket (Remark "Approximate solvers")
    rd = step(prec, want_phi=True, wirebasket="diagonal")
    errd = np.linalg.norm(rd["phi"] - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
    rd["M"].close()
    rd["problem"].close()
    diag_step = {"t_step_s": rd["t_step"], "t_precond_s": rd["t_precond"], "t_solve_s": rd["t_solve"],
                 "iters": rd["iters"], "relerr_max": float(errd.max()),
                 "solves_per_s": int((errd <= 1e-8).sum()) / rd["t_step"]}
    log("bench: diagonal wire basket: step %.3fs precond %.4f solve %.3f iters %s" %
        (rd["t_step"], rd["t_precond"], rd["t_solve"], rd["iters"][:4]))

    # the same step with host buffers (mesh uploaded, solutions downloaded in the step): the
    # PCIe-inclusive rate, reported beside the value, never as it
    t_h0 = time.perf_counter()
    n_h, solved_h = 2, 0
    for _ in range(n_h):
        rh = step(prec, want_phi=True)
        errh = np.linalg.norm(rh["phi"] - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        solved_h += int((errh <= 1e-8).sum())
        rh["M"].close()
        rh["problem"].close()
    t_h = time.perf_counter() - t_h0
    host_io = {"steps": n_h, "ms_per_step": t_h / n_h * 1e3, "solves_per_s": solved_h / t_h}
    log("bench: host-buffer steps (PCIe-inclusive): %.1f ms per step" % (t_h / n_h * 1e3))

    nt = pinfo["n_tri"]
    pairs = nt * (nt + 1) // 2
    t_asm = float(np.mean([r["t_assemble"] for r in res]))
    t_far = float(np.mean([r["t_far"] for r in res]))
    far_pairs = pairs - pinfo["n_near_pairs"]
    far_tflops = far_pairs * EVALS_PER_FAR_PAIR * FLOPS_PER_EVAL / t_far / 1e12
    mv = {**matvec_rates(N, 8, t64_1, "fp64_k1"), **matvec_rates(N, 8, t64_16, "fp64_k16")}
    if mixed:
        mv.update(matvec_rates(N, 4, t32_1, "fp32_k1"))
        mv.update(matvec_rates(N, 4, t32_16, "fp32_k16"))
    lat = sorted(r["t_step"] for r in res)
    roofline = {
        "kernel": "k_far",
        "bound": "alu",
        "achieved": round(far_tflops, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(far_tflops / PEAK_FP64_TFLOPS, 4),
        "traffic": load_traffic("k_far", args.workload),
        "per_launch": "%d far pairs x %d evaluations x %.4f flops" % (far_pairs, EVALS_PER_FAR_PAIR, FLOPS_PER_EVAL),
        "avg_launch_s": t_far,
    }
    out = {
        "metric": "PCG solves/s + p50/p99 latency at rel.err 1e-8; pair-integrals/s; matvec GB/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %s; %d right-hand sides per step (block PCG), %s PCG to relative "
                               "residual %.0e, rel.err <= 1e-8 vs FP64 reference" %
                               (args.workload, w.description, args.k, "mixed-precision (FP32 products, reliable FP64 residual updates)" if mixed else "FP64",
                                args.tol),
                   "n_dofs": N, "n_tri": nt, "k": args.k, "precision": args.precision,
                   "patches": ref["precond_sizes"],
                   "io": "mesh and solutions resident in device memory (bem_assemble_dev, bem_pcg_solve_dev); "
                         "the host-buffer rate is pcie_inclusive"},
        "roofline": roofline,
        "pair_integrals_per_s": pairs / t_asm,
        "pair_integrals_per_s_far_kernel": far_pairs / t_far,
        "latency_s": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]},
        "phases_s": {k_: float(np.mean([r[k_] for r in res])) for k_ in
                     ("t_step", "t_assemble", "t_host", "t_far", "t_near", "t_contract", "t_precond", "t_solve")},
        "iters": res[-1]["iters"],
        "outer_iters": res[-1]["outer"],
        "relerr_max": max(max(r["relerr"]) for r in res),
        "matvec": mv,
        "fp64_compare": fp64_step,
        "diagonal_wirebasket": diag_step,
        "pcie_inclusive": host_io,
    }
    if not args.no_potential:
        out["double_layer"] = double_layer_leg(lib, w, ctx)
    if not args.no_planar:
        out["planar"] = planar_leg(lib, meshes, ctx)
    if not args.no_kappa:
        log("bench: condition-number study")
        out["kappa_study"] = kappa_study(lib, meshes, ctx)
    if not args.no_large and args.workload != "crossed192":
        log("bench: crossed192 leg")
        out["crossed192"] = large_leg(lib, meshes, ctx)
    if args.serve_requests > 0:
        log("bench: serving stream (%d requests, load %.2f)" % (args.serve_requests, args.serve_load))
        out["serving"] = serving_leg(lib, meshes, ctx, args.serve_requests, args.serve_load)
    if not args.no_cpu_baseline:
        log("bench: oracle on host cores (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(w, args.k, int(np.mean(res[-1]["iters"])), pinfo, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
