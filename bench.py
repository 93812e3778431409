#!/usr/bin/env python3
"""Benchmark of the whole hot path on one MI355X.

One step = one pass of the path over one batch of synthetic input: host mesh analysis and near
list, device assembly of W (far 7x7 tiles, Duffy near kernels, contraction, FP32 copy), right-hand
sides, preconditioner set-up (block inverses, coarse Galerkin matrix), and the mixed-precision PCG
solve of k right-hand sides to relative residual tol.  The headline workload is crossed192 (three
perpendicular unit squares, h = 1/192: 221,184 triangles, 110,017 dofs, the pair matrix built in
panels), the largest configuration that fits one GPU.  Every solved column is checked against an
FP64 GPU solve of the same system at relative residual 1e-13 (self-consistency); only columns
within 1e-8 count.  The oracle's sampled residual rows of the same solutions ride along in the
CPU-baseline leg (parity).

Prints one JSON line (see the "metric"/"value" keys); per-phase timings, matvec HBM rates, the
roofline of the dominant kernel, side legs (crossed96, the unit square and the book, the book's
condition-number study, serving, the paper's experiments) and the oracle timed on the host cores
ride along.
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
GOLDEN = os.path.join(ROOT, "tests", "golden")

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
# algorithmic FP64 flops of one far-field kernel evaluation w / |x - y|: 3 subtractions and 3
# multiply-adds for |x - y|^2, one multiply-add into the sum (the reciprocal square root not
# counted); a multiply-add counts 2
FLOPS_PER_EVAL = 11.0
# the same evaluation as the far kernel issues it in its gfx950 ISA (direct form: 3 add, 3 mul,
# 4.14 FMA, including the Newton step of v_rsq_f64), reported beside the algorithmic rate
ISA_FLOPS_PER_EVAL = 14.0 + 2.0 / 7.0
EVALS_PER_FAR_PAIR = 49


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def far_kernel_source_hash():
    """Hash of the far-field pass's own source text (its constants, the one-shot and the panel
    kernels, through the panel kernel's closing brace, and the panel tile list's order), so that
    counters taken on an older version are not reported."""
    src = open(os.path.join(ROOT, "paper_2310_09204_amd", "csrc", "assemble.hip")).read()
    a = src.index("constexpr int kGrp")
    b = src.index("\n}\n", src.index("void k_far_rect(", a)) + 3
    c = src.index("constexpr int kRowGroup")
    d = src.index("\n}\n", src.index("void k_rect_tiles(", c)) + 3
    return hashlib.sha256((src[a:b] + src[c:d]).encode()).hexdigest()[:16]


def symv_bytes(N, size, ks):
    """HBM bytes of one symmetric product (any number of columns up to 16): the upper block triangle of W
    (64 x 64 blocks) plus the block-row partials written and read back (super-blocks of ks blocks, the
    problem's tuned value; one partial of 64 rows x 16 columns per block row and super-tile, plus one)."""
    nb = (N + 63) // 64
    nst = (nb + ks - 1) // ks
    return nb * (nb + 1) // 2 * 64 * 64 * size + 2 * nb * (nst + 1) * 1024 * size


def matvec_rates(N, size, t, key, ks):
    """A product's time, its algorithmic HBM bytes (upper block triangle + partials), the rate and
    its fraction of the 8 TB/s peak."""
    b = symv_bytes(N, size, ks)
    return {key + "_ms": t * 1e3, key + "_bytes": b, key + "_hbm_GBs": b / t / 1e9,
            key + "_hbm_frac": b / t / 1e9 / PEAK_HBM_GBS}


def load_traffic(kernel, workload, launches):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if the kernel source is
    unchanged since the counters were taken and the step had the same number of launches (panels);
    else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(kernel, {}).get(workload)
        if not e or e.get("source_hash") != far_kernel_source_hash():
            return None
        if int(e.get("launches_per_step", 1)) != int(launches):
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def input_hash(w):
    h = hashlib.sha256()
    for a in (w.mesh.vertices, w.mesh.triangles, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles,
              w.coarse_of_triangle, w.g):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def golden(name, w):
    """The oracle's stored results for workload w (tests/golden/<name>_reference.npz), or None if the
    file is absent or was written for other inputs."""
    path = os.path.join(GOLDEN, name + "_reference.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    return ref if str(ref["input_hash"]) == input_hash(w) else None


def percentile(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]


# ---------------------------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores
# ---------------------------------------------------------------------------------------------

def cpu_baseline(w, k, iters, gpu_info, precond_sizes, budget_s, phi_checks):
    """The oracle as it stands, timed on the host cores on bounded samples of this workload and
    scaled to one step (assembly, preconditioner set-up, k PCG solves of `iters` iterations).

    Measured in full: the oracle's mesh analysis (sectors, dofs, jump coefficients), its dof
    classification and its coarse prolongation.  Sampled and scaled by their work units:
      * pair integrals: every column of the rows of I that the stars of a window of dofs touch
        (oracle_I_rows), scaled to the N_T rows the oracle's assembly computes;
      * contraction: the oracle's contraction of that panel into the window's rows
        (oracle_W_accumulate), scaled by star entries;
      * set-up: Cholesky factorizations (the oracle's scipy cho_factor) of SPD stand-ins of the
        workload's block sizes (a sample of faces, the whole wire basket, the coarse block), and
        the coarse product R_H W on a slab of rows of a stand-in W;
      * solve: the oracle's PCG is one column at a time; per iteration its dense product W p
        (numpy, on a slab of rows of a stand-in W) and one application of the block solves
        (scipy cho_solve on the stand-in factors, plus R_H^T and R_H).
    Parity rides along: the oracle's rows of W for a few seeded dofs (every q = 8 origin dof among
    them) give the residual rows (L - W phi)_S of the GPU solutions in phi_checks."""
    import scipy.linalg as sla
    from oracle.assemble import I_rows, W_accumulate, W_rows, _JumpCSR, rhs
    from oracle.precond import classify_dofs, coarse_prolongation
    from oracle.topology import Topology

    m = w.mesh
    V = np.ascontiguousarray(m.vertices, dtype=np.float64)
    T = np.ascontiguousarray(m.triangles, dtype=np.int32)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)
    out = {"kind": "oracle", "unit": "solves/s", "cores": threads}

    t0 = time.perf_counter()
    topo = Topology(V, T)
    t_topo = time.perf_counter() - t0
    log("bench: oracle mesh analysis %.1f s" % t_topo)
    nt, N = topo.nt, topo.N
    assert N == int(gpu_info["n_dofs"])
    c = _JumpCSR(topo)

    # pair integrals and contraction on the rows of a dof window's stars, grown until it has taken
    # about a third of the budget
    d0 = N // 3
    size, t_rows, rows_done, t_acc, entries_done, tries = 16, 0.0, 0, 0.0, 0, 0
    while (t_rows < 0.35 * budget_s or rows_done == 0) and size <= 4096 and tries < 1000:
        tries += 1
        d0 = min(d0, N - 1)
        d1 = min(N, d0 + size)
        tris = c.dof_tri[c.dof_ptr[d0]:c.dof_ptr[d1]]
        r0, r1 = int(tris.min()), int(tris.max()) + 1
        if r1 - r0 > max(16 * size, 2048) and tries < 999:   # the window reaches distant triangles: move on
            d0 = (d0 + size) % max(1, N - size)
            continue
        ta = time.perf_counter()
        I = I_rows(V, T, r0, r1 - r0, 10)
        tb = time.perf_counter()
        W_accumulate(topo, r0, I, d0, d1, c)
        tc = time.perf_counter()
        del I
        t_rows += tb - ta
        rows_done += r1 - r0
        t_acc += tc - tb
        entries_done += int(c.dof_ptr[d1] - c.dof_ptr[d0])
        d0 = d1
        size *= 2
    t_pairs = t_rows / rows_done * nt
    log("bench: oracle %d rows of I in %.1f s, contraction of %d entries in %.2f s" % (rows_done, t_rows, entries_done, t_acc))
    t_contract = t_acc / entries_done * len(c.dof_tri)

    # set-up: classification and prolongation in full; factorizations on SPD stand-ins
    t0 = time.perf_counter()
    faces, wb = classify_dofs(topo, w.patch_of_triangle)
    t_classify = time.perf_counter() - t0
    t0 = time.perf_counter()
    RH, _ = coarse_prolongation(topo, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
    t_prolong = time.perf_counter() - t0
    nH = RH.shape[0]

    def spd(n):
        A = rng.standard_normal((n, n))
        return (A + A.T) / 2 + 2.0 * np.sqrt(n) * np.eye(n)

    face_sizes = [len(f) for f in faces]
    sample = rng.choice(len(face_sizes), min(16, len(face_sizes)), replace=False)
    fac_faces, t_ff = [], 0.0
    for i in sample:
        A = spd(face_sizes[i])
        t0 = time.perf_counter()
        fac_faces.append(sla.cho_factor(A, lower=True))
        t_ff += time.perf_counter() - t0
    t_face_factor = t_ff / len(sample) * len(face_sizes)
    A = spd(len(wb))
    t0 = time.perf_counter()
    fac_wb = sla.cho_factor(A, lower=True)
    t_wb_factor = time.perf_counter() - t0
    del A
    AH = spd(nH)
    t0 = time.perf_counter()
    fac_H = sla.cho_factor(AH, lower=True)
    t_coarse_factor = time.perf_counter() - t0
    slab = min(N, 1024)
    Wslab = rng.standard_normal((slab, N))
    t0 = time.perf_counter()
    RH[:, :slab] @ Wslab            # one slab of the coarse product R_H W (then Z R_H^T, n_H^2 N: small)
    t_coarse_product = (time.perf_counter() - t0) * (N / slab)
    log("bench: oracle set-up samples done (prolongation %.1f s)" % t_prolong)
    t_setup = t_classify + t_prolong + t_face_factor + t_wb_factor + t_coarse_factor + t_coarse_product

    # solve: per column and iteration one dense product and one preconditioner application
    p = rng.standard_normal(N)
    reps, t_mv = 0, 0.0
    while t_mv < 0.05 * budget_s and reps < 50:
        t0 = time.perf_counter()
        Wslab @ p
        t_mv += time.perf_counter() - t0
        reps += 1
    t_matvec = t_mv / reps * (N / slab)
    del Wslab
    r = rng.standard_normal(N)
    t0 = time.perf_counter()
    for i, f in zip(sample, fac_faces):
        sla.cho_solve(f, r[:face_sizes[i]])
    t_fs = (time.perf_counter() - t0) / len(sample) * len(face_sizes)
    t0 = time.perf_counter()
    sla.cho_solve(fac_wb, r[:len(wb)])
    RH.T @ sla.cho_solve(fac_H, RH @ r)
    t_apply = t_fs + time.perf_counter() - t0
    t_solve = k * iters * (t_matvec + t_apply)

    t_assembly = t_topo + t_pairs + t_contract
    t_step = t_assembly + t_setup + t_solve
    out.update({
        "value": k / t_step,
        "sample": "oracle mesh analysis, dof classification and coarse prolongation in full; %d rows of the "
                  "pair-integral matrix (all %d columns, oracle_I_rows) and their contraction into %d star "
                  "entries (oracle_W_accumulate), scaled to %d rows / %d entries; Cholesky (scipy) of SPD "
                  "stand-ins for %d of %d faces, the %d-dof wire basket and the %d-dof coarse block; the "
                  "coarse product and the PCG's dense product on a %d-row slab of a stand-in W, and one "
                  "application of the block solves; %d right-hand sides x %d PCG iterations, one column "
                  "at a time as the oracle's PCG runs"
                  % (rows_done, nt, entries_done, nt, len(c.dof_tri), len(sample), len(face_sizes), len(wb), nH,
                     slab, k, iters),
        "t_step_s": t_step, "t_assembly_s": t_assembly, "t_setup_s": t_setup, "t_solve_s": t_solve,
        "t_mesh_analysis_s": t_topo, "t_pair_integrals_s": t_pairs, "t_contraction_s": t_contract,
        "t_setup_parts_s": {"classify": t_classify, "prolongation": t_prolong, "face_factors": t_face_factor,
                            "wirebasket_factor": t_wb_factor, "coarse_factor": t_coarse_factor,
                            "coarse_product": t_coarse_product},
        "t_matvec_s": t_matvec, "t_precond_apply_s": t_apply,
        # the oracle's assembly computes all N_T^2 ordered pairs (full rows of I)
        "pair_integrals_computed_per_s": rows_done * nt / t_rows,
        "pair_integrals_per_s": nt * (nt + 1) / 2 / t_assembly,
        "matvec_GBs": N * N * 8 / t_matvec / 1e9,
    })

    # parity: oracle residual rows of the GPU solutions
    qd = np.array([topo.q[v] for v, j in topo.dofs])
    special = np.nonzero(qd == 8)[0]
    S = np.unique(np.concatenate([special, rng.choice(N, 32, replace=False)])).astype(np.int64)
    t0 = time.perf_counter()
    Wo = W_rows(V, T, S, topo=topo, near_order=10)
    L = rhs(topo, w.g).T
    res = {}
    for name, phi in phi_checks.items():
        rr = L[:, S] - phi @ Wo.T
        res[name] = float((np.linalg.norm(rr, axis=1) / np.linalg.norm(L[:, S], axis=1)).max())
    out["oracle_residual_rows"] = {"rows": len(S), "max_relative": res, "t_s": time.perf_counter() - t0}
    log("bench: oracle residual rows %s" % res)
    return out


# ---------------------------------------------------------------------------------------------
# the timed workload
# ---------------------------------------------------------------------------------------------

def timed_workload(lib, meshes, ctx, name, k, steps, warmup, tol, mixed, extras=True):
    """Warm-up and timed steps of `name` with k right-hand sides (mesh and solutions resident in
    device memory), an FP64 GPU reference solve at tol 1e-13 beside them, and untimed extras: the
    FP64-only solve, the diagonal wire basket, the host-buffer (PCIe-inclusive) step, the matvec
    rates.  Returns (summary dict, solutions of the last timed step, reference solutions)."""
    w = meshes.workload(name, seed=0, k=k)
    m = w.mesh
    prec = lib.FP32_REFINE if mixed else lib.FP64
    ctx.release_cached()
    d_mesh = (lib.DeviceArray(np.asarray(m.vertices, dtype=np.float64)),
              lib.DeviceArray(np.asarray(m.triangles, dtype=np.int32)))

    def step(precision, keep=False, tol=tol, wirebasket="exact", device_out=None):
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
               "t_host": pinfo["t_host_s"], "iters": [i["iters"] for i in info],
               "outer": [i["outer_iters"] for i in info], "rc": rc, "info": pinfo, "precond_sizes": M.sizes(),
               "phi": phi}
        if keep:
            out["problem"], out["M"] = p, M
        else:
            M.close()
            p.close()
        return out

    # FP64 reference (not timed), the FP64-only solve and the FP64 product rates on the same system
    log("bench: %s FP64 reference solve (tol 1e-13)" % name)
    ref = step(lib.FP64, keep=True, tol=1e-13)
    phi_ref = ref["phi"]
    pinfo = ref["info"]
    N = pinfo["n_dofs"]
    pref, Mref = ref["problem"], ref["M"]
    tun = pref.tuning
    fp64_solve = None
    if extras and mixed:
        t0 = time.perf_counter()
        phi64, info64, _ = pref.solve(g=w.g, precond=Mref, tol=tol, precision=lib.FP64)
        t_s64 = time.perf_counter() - t0
        e64 = np.linalg.norm(phi64 - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        fp64_solve = {"t_solve_s": t_s64, "iters": [i["iters"] for i in info64], "relerr_max": float(e64.max()),
                      "t_step_s": ref["t_assemble"] + ref["t_precond"] + t_s64}
    t64_1 = pref.bench_matvec(fp32=False, k=1, reps=5)
    t64_16 = pref.bench_matvec(fp32=False, k=16, reps=3)
    Mref.close()
    pref.close()
    ctx.release_cached()

    # one device buffer per timed step for its solutions, allocated before the timed region
    d_out = [lib.DeviceArray(shape=(w.g.shape[0], N)) for _ in range(max(steps, 1))]
    for i in range(warmup):
        log("bench: %s warm-up step %d" % (name, i))
        r = step(prec, device_out=d_out[0])
        log("bench: %s warm-up %.3fs" % (name, r["t_step"]))
    ctx.synchronize()
    res = []
    t_begin = time.perf_counter()
    for i in range(steps):
        res.append(step(prec, device_out=d_out[i]))
    ctx.synchronize()
    elapsed = time.perf_counter() - t_begin
    phis = [d.get() for d in d_out[:steps]]
    for d in d_out + list(d_mesh):
        d.close()
    for i, (r, phi) in enumerate(zip(res, phis)):
        err = np.linalg.norm(phi - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        r["relerr"] = err.tolist()
        r["solved"] = int((err <= 1e-8).sum())
        log("bench: %s step %d %.3fs asm %.3f (host %.3f far %.3f near %.4f contract %.3f) precond %.3f solve %.3f "
            "iters %s relerr max %.2e" % (name, i, r["t_step"], r["t_assemble"], r["t_host"], r["t_far"], r["t_near"],
                                          r["t_contract"], r["t_precond"], r["t_solve"], r["iters"][:4], max(r["relerr"])))
    solved = sum(r["solved"] for r in res)
    nt = pinfo["n_tri"]
    pairs = nt * (nt + 1) // 2
    far_pairs = pairs - pinfo["n_near_pairs"]
    # panels of the timed steps' problems (the FP64 reference, without the FP32 copy, has room for
    # larger ones)
    panels = int(res[-1]["info"]["n_pair_panels"])
    launches = max(1, panels)
    t_far = float(np.mean([r["t_far"] for r in res]))
    far_kernel = "k_far_rect" if panels > 0 else "k_far"
    far_tflops = far_pairs * EVALS_PER_FAR_PAIR * FLOPS_PER_EVAL / t_far / 1e12
    out = {
        "workload": name, "description": w.description, "n_dofs": N, "n_tri": nt, "k": k,
        "precision": "mixed" if mixed else "fp64", "tol": tol,
        "pair_panels": panels,
        "steps": steps, "warmup": warmup, "elapsed_s": elapsed,
        "value": solved / elapsed, "ms_per_step": elapsed / steps * 1e3,
        "latency_s": {"p50": percentile([r["t_step"] for r in res], 0.5),
                      "p99": percentile([r["t_step"] for r in res], 0.99)},
        "phases_s": {k_: float(np.mean([r[k_] for r in res])) for k_ in
                     ("t_step", "t_assemble", "t_host", "t_far", "t_near", "t_contract", "t_precond", "t_solve")},
        "iters": res[-1]["iters"], "outer_iters": res[-1]["outer"],
        "relerr_max": max(max(r["relerr"]) for r in res),
        "relerr_reference": "FP64 GPU PCG of the same system at relative residual 1e-13 (self-consistency; "
                            "oracle parity: cpu_baseline.oracle_residual_rows and the GPU tests)",
        "patches": ref["precond_sizes"],
        # pairs per second of the assembly's device time (the call returns before it ends)
        "pair_integrals_per_s": pairs / float(np.mean([r["t_far"] + r["t_near"] + r["t_contract"] for r in res])),
        "pair_integrals_per_s_far_kernel": far_pairs / t_far,
        "roofline": {
            "kernel": far_kernel, "bound": "alu",
            "achieved": round(far_tflops, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(far_tflops / PEAK_FP64_TFLOPS, 4),
            "traffic": load_traffic(far_kernel, name, launches),
            "per_launch": "%d far pairs x %d evaluations x %.0f flops over %d launch(es)"
                          % (far_pairs, EVALS_PER_FAR_PAIR, FLOPS_PER_EVAL, launches),
            "launches": launches, "avg_launch_s": t_far / launches,
            "isa_tflops": round(far_pairs * EVALS_PER_FAR_PAIR * ISA_FLOPS_PER_EVAL / t_far / 1e12, 3),
        },
        "fp64_solve": fp64_solve,
        "tuning": tun,
    }
    ks64, ks32 = tun["symv_blocks_fp64"], tun["symv_blocks_fp32"]
    mv = {**matvec_rates(N, 8, t64_1, "fp64_k1", ks64), **matvec_rates(N, 8, t64_16, "fp64_k16", ks64)}
    phi_last = phis[-1]
    if extras:
        # the same step with host buffers (mesh uploaded, solutions downloaded): the PCIe-inclusive
        # rate, reported beside the value, never as it; its problem then serves the FP32 product
        # rates and the diagonal wire basket
        rh = step(prec, keep=True)
        errh = np.linalg.norm(rh["phi"] - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        out["pcie_inclusive"] = {"ms_per_step": rh["t_step"] * 1e3,
                                 "solves_per_s": int((errh <= 1e-8).sum()) / rh["t_step"]}
        p, M = rh["problem"], rh["M"]
        M.close()
        if mixed:
            t32_1 = p.bench_matvec(fp32=True, k=1, reps=5)
            t32_16 = p.bench_matvec(fp32=True, k=16, reps=3)
            mv.update(matvec_rates(N, 4, t32_1, "fp32_k1", ks32))
            mv.update(matvec_rates(N, 4, t32_16, "fp32_k16", ks32))
        # both set-ups timed on the finished problem; the diagonal step is the timed step with the
        # exact set-up and solve replaced by these (the timed steps' t_precond also holds the end of
        # the assembly's device work)
        ctx.synchronize()
        te0 = time.perf_counter()
        Me = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                                factor_fp32=mixed)
        te1 = time.perf_counter()
        Me.close()
        t0 = time.perf_counter()
        Md = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                                factor_fp32=mixed, wirebasket="diagonal")
        t1 = time.perf_counter()
        phid, infod, _ = p.solve(g=w.g, precond=Md, tol=tol, precision=prec)
        t2 = time.perf_counter()
        errd = np.linalg.norm(phid - phi_ref, axis=1) / np.linalg.norm(phi_ref, axis=1)
        ph = out["phases_s"]
        t_stepd = ph["t_step"] - (te1 - te0) - ph["t_solve"] + (t1 - t0) + (t2 - t1)
        out["exact_wirebasket_setup_s"] = te1 - te0
        out["diagonal_wirebasket"] = {"t_precond_s": t1 - t0, "t_solve_s": t2 - t1, "t_step_s": t_stepd,
                                      "iters": [i["iters"] for i in infod], "relerr_max": float(errd.max()),
                                      "solves_per_s": int((errd <= 1e-8).sum()) / t_stepd}
        Md.close()
        p.close()
        ctx.release_cached()
        if fp64_solve is not None:
            fp64_solve["solves_per_s"] = int(k) / fp64_solve["t_step_s"] if fp64_solve["relerr_max"] <= 1e-8 else 0.0
    out["matvec"] = mv
    # at crossed96 the oracle's exact solution of the first two columns is stored: parity
    g = golden(name, meshes.workload(name, seed=0, k=2))
    if g is not None:
        phis_o = g["phi"]
        e = np.linalg.norm(phi_last[:2] - phis_o, axis=1) / np.linalg.norm(phis_o, axis=1)
        out["oracle_relerr_max"] = float(e.max())
    return out, w, phi_last, phi_ref


# ---------------------------------------------------------------------------------------------
# side legs
# ---------------------------------------------------------------------------------------------

def small_configs_leg(lib, meshes, ctx):
    """The unit square (16 x 16 cells) and the three-page book (h = 1/48) in FP64: PCG and CG
    iteration counts at relative residual 1e-10 next to the oracle's, solves/s of whole steps
    (assembly, set-up, PCG to 1e-13) counting columns within 1e-10 of the oracle's Phi*, and
    pair-integrals/s; then kappa(P_ad W) of the book at H/h = 4 .. 24 next to the oracle's."""
    out = {}
    for name, k, reps in (("square16", 1, 20), ("book48", 3, 5)):
        w = meshes.workload(name, seed=0, k=k)
        ref = golden(name, w)
        if ref is None:
            raise RuntimeError("tests/golden/%s_reference.npz missing or stale" % name)
        m = w.mesh
        p = lib.Problem(ctx, m.vertices, m.triangles, near_order=10)
        M = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle)
        _, ip, _ = p.solve(g=w.g, precond=M, tol=1e-10)
        _, ic, _ = p.solve(g=w.g, precond=None, tol=1e-10)
        M.close()
        p.close()
        times, solved, worst, t_asm = [], 0, 0.0, []
        for rep in range(reps + 1):             # the first repetition warms up
            t0 = time.perf_counter()
            p = lib.Problem(ctx, m.vertices, m.triangles, near_order=10)
            t1 = time.perf_counter()
            M = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles,
                                   w.coarse_of_triangle)
            phi, _, _ = p.solve(g=w.g, precond=M, tol=1e-13)
            t2 = time.perf_counter()
            M.close()
            p.close()
            e = np.linalg.norm(phi - ref["phi"], axis=1) / np.linalg.norm(ref["phi"], axis=1)
            worst = max(worst, float(e.max()))
            if rep > 0:
                times.append(t2 - t0)
                t_asm.append(t1 - t0)
                solved += int((e <= 1e-10).sum())
        nt = m.nt
        out[name] = {"n_dofs": int(ref["phi"].shape[1]), "n_tri": nt, "k": k, "steps": reps,
                     "ms_per_step": float(np.mean(times)) * 1e3, "solves_per_s": solved / float(np.sum(times)),
                     "relerr_vs_oracle_max": worst,
                     "pcg_iters": [i["iters"] for i in ip], "cg_iters": [i["iters"] for i in ic],
                     "oracle_pcg_iters": ref["pcg_iters"].tolist(), "oracle_cg_iters": ref["cg_iters"].tolist(),
                     "pair_integrals_per_s": nt * (nt + 1) / 2 / float(np.mean(t_asm))}
        log("bench: %s %.2f ms per step, PCG %s CG %s (oracle %s %s), err %.1e" %
            (name, out[name]["ms_per_step"], out[name]["pcg_iters"], out[name]["cg_iters"],
             out[name]["oracle_pcg_iters"], out[name]["oracle_cg_iters"], worst))
    # the book's condition-number growth (Thm. main) at fixed h = 1/48
    w = meshes.workload("book48", seed=0, k=1)
    ref = golden("book48", meshes.workload("book48", seed=0, k=3))
    m = w.mesh
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=10)
    rows = []
    for j, r in enumerate(ref["kappa_ratio"].tolist()):
        patches = meshes.grid_patches(m, r)
        cm, par = meshes.coarse_mesh(m, r)
        M = lib.Preconditioner(p, patches, cm.vertices, cm.triangles, par)
        _, info, _ = p.solve(g=w.g, precond=M, tol=1e-12)
        s = M.sizes()
        M.close()
        kp = info[0]["est_cond"]
        rows.append({"H_over_h": r, "faces": s["n_faces"], "wb": s["n_wb"], "coarse": s["n_coarse"],
                     "kappa_pad": kp, "kappa_over_log2": kp / (1 + np.log(r)) ** 2, "pcg_iters": info[0]["iters"],
                     "oracle_kappa_pad": float(ref["kappa_pad"][j]), "oracle_pcg_iters": int(ref["kappa_iters"][j])})
        log("bench: book48 H/h=%d kappa %.3f (oracle %.3f) iterations %d" % (r, kp, rows[-1]["oracle_kappa_pad"],
                                                                            info[0]["iters"]))
    _, info, _ = p.solve(g=w.g, precond=None, tol=1e-12)
    p.close()
    out["book48_kappa"] = {"rows": rows, "kappa_W": info[0]["est_cond"], "oracle_kappa_W": float(ref["kappa_W"])}
    return out


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

    Capacity is measured first by submitting the whole stream at once (after one untimed burst
    that warms the buffer pool; each replay starts a new server, so every geometry is assembled
    and set up again inside the timed region); the timed replay then scales the seeded arrival
    times to `load` x capacity.  Latency is submit -> completion as the
    server measures it; solves/s counts right-hand sides within rel.err 1e-8 of an FP64 solve of
    the same request (computed after the stream, not timed).  Each latency splits into the wait
    before the request's columns start in a block PCG (queueing, plus assembly and set-up of a
    geometry that was not resident) and the solve after it."""
    # The previous legs' buffers go back to the driver, and an untimed burst then fills the buffer
    # pool with the stream's own sizes, as a server that has run for a while holds them.  Once a
    # process has written a few hundred GB of device memory, handing memory back to the driver
    # gets slow (hipFree of 48 GiB: about 1 s, against 2 ms before) and so does the work right
    # after it: a server started from an empty pool after the crossed192 legs timed that, at a
    # third of the rate it reaches in a fresh process.
    ctx.release_cached()
    reqs = meshes.serving_stream(seed, n_requests, rate=1.0)    # arrival times for rate 1/s
    _replay(lib, reqs, ctx, 0.0, max_inflight)
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
    lat = [res[1][0]["t_total_s"] for res in results]
    wait = [res[1][0]["t_start_s"] for res in results]
    n_dofs = [int(res[0].shape[1]) for res in results]
    slowest = sorted(range(len(reqs)), key=lambda i: -lat[i])[:3]
    return {
        "requests": len(reqs), "failed_requests": len(failed),
        "direct_launch_requests": sum(1 for res in results if res[2] >= 0 and res[1][0]["graph"] == 0),
        "rhs": total, "rhs_within_1e-8": solved, "relerr_max": worst,
        "capacity_requests_per_s": capacity, "load": load, "arrival_rate_per_s": rate,
        "max_inflight": max_inflight,
        "solves_per_s": solved / t_run,
        "latency_s": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99)},
        "start_wait_s": {"p50": percentile(wait, 0.5), "p99": percentile(wait, 0.99)},
        "solve_after_start_s": {"p50": percentile([a - b for a, b in zip(lat, wait)], 0.5),
                                "p99": percentile([a - b for a, b in zip(lat, wait)], 0.99)},
        "slowest": [{"request": i, "n_dofs": n_dofs[i], "k": int(reqs[i].g.shape[0]), "mixed": bool(reqs[i].mixed),
                     "latency_s": lat[i], "start_wait_s": wait[i]} for i in slowest],
        "n_dofs_range": [min(n_dofs), max(n_dofs)],
        "mixed_requests": int(sum(r.mixed for r in reqs)),
        "server": stats,
    }


def double_layer_leg(lib, meshes, ctx, m_targets=16384, k=16):
    """Double-layer potential (Lemma repDL) of k crossed96 solutions at seeded targets in [-1, 1]^3
    at least 0.05 (about 5 h) from every panel plane: evaluations (target x Gauss point) per second
    and the FP64 rate, counting 16 + 2 k flops per evaluation (distance 8, Newton step 4, cube 2,
    normal projection 2, one FMA per column; the reciprocal square root not counted)."""
    w = meshes.workload("crossed96", seed=0, k=k)
    m = w.mesh
    p = lib.Problem(ctx, m.vertices, m.triangles, precision=lib.FP32_REFINE, near_order=10)
    M = lib.Preconditioner(p, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                           factor_fp32=True)
    phi, _, _ = p.solve(g=w.g, precond=M, tol=1e-10, precision=lib.FP32_REFINE)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="crossed192", help="crossed192 (headline) or crossed96")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="time budget of the oracle's pair-integral sample (the rest of the baseline adds to it)")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests in the serving-stream leg (0 skips it)")
    ap.add_argument("--no-side", action="store_true", help="skip the crossed96 side leg")
    ap.add_argument("--no-small", action="store_true", help="skip the unit square / book leg")
    ap.add_argument("--no-kappa", action="store_true", help="skip the two-triangle condition-number study")
    ap.add_argument("--no-potential", action="store_true", help="skip the double-layer potential leg")
    ap.add_argument("--no-planar", action="store_true", help="skip the two-dimensional experiments")
    ap.add_argument("--headline-only", action="store_true", help="only the timed workload (profiling runs)")
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
    if args.headline_only:
        args.no_cpu_baseline = args.no_side = args.no_small = args.no_kappa = True
        args.no_potential = args.no_planar = True
        args.serve_requests = 0

    from paper_2310_09204_amd import lib, meshes

    mixed = args.precision == "mixed"
    log("bench: workload %s k=%d precision=%s" % (args.workload, args.k, args.precision))
    ctx = lib.Context(0)
    head, w, phi_last, phi_ref = timed_workload(lib, meshes, ctx, args.workload, args.k, args.steps, args.warmup,
                                                args.tol, mixed, extras=not args.headline_only)
    out = {
        "metric": "PCG solves/s + p50/p99 latency at rel.err 1e-8; pair-integrals/s; matvec GB/s",
        "value": round(head["value"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %s; %d right-hand sides per step (block PCG), %s PCG to relative "
                               "residual %.0e, rel.err <= 1e-8 vs an FP64 solve at 1e-13" %
                               (args.workload, w.description, args.k,
                                "mixed-precision (FP32 products, reliable FP64 residual updates)" if mixed else "FP64",
                                args.tol),
                   "n_dofs": head["n_dofs"], "n_tri": head["n_tri"], "k": args.k, "precision": args.precision,
                   "patches": head["patches"], "pair_panels": head["pair_panels"],
                   "tuning": {"table": "paper_2310_09204_amd/tuning/gfx950.json" if ctx.tuning else "defaults",
                              "applied": head["tuning"]},
                   "io": "mesh and solutions resident in device memory (bem_assemble_dev, bem_pcg_solve_dev); "
                         "the host-buffer rate is pcie_inclusive"},
        "roofline": head["roofline"],
        "latency_s": head["latency_s"],
        "pair_integrals_per_s": head["pair_integrals_per_s"],
        "matvec": head["matvec"],
        "headline": head,
    }
    if not args.no_side and args.workload != "crossed96":
        log("bench: crossed96 side leg")
        side, _, _, _ = timed_workload(lib, meshes, ctx, "crossed96", args.k, args.steps, 1, args.tol, mixed)
        out["crossed96"] = side
    if not args.no_small:
        log("bench: unit square and book (FP64)")
        out["small_configs"] = small_configs_leg(lib, meshes, ctx)
    if not args.no_potential:
        out["double_layer"] = double_layer_leg(lib, meshes, ctx)
    if not args.no_planar:
        out["planar"] = planar_leg(lib, meshes, ctx)
    if not args.no_kappa:
        log("bench: condition-number study")
        out["kappa_study"] = kappa_study(lib, meshes, ctx)
    if args.serve_requests > 0:
        log("bench: serving stream (%d requests, load %.2f)" % (args.serve_requests, args.serve_load))
        out["serving"] = serving_leg(lib, meshes, ctx, args.serve_requests, args.serve_load)
    ctx.close()
    if not args.no_cpu_baseline:
        log("bench: oracle on host cores (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(w, args.k, int(round(np.mean(head["iters"]))), head, head["patches"],
                                           args.cpu_seconds, {"mixed": phi_last, "fp64_reference": phi_ref})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
