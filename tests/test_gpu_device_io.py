"""Device-resident inputs and outputs through the C-ABI: bem_assemble_dev (the kernels read the
caller's device copy of the mesh) and bem_pcg_solve_dev (the solution stays in device memory)
give exactly what the host-buffer entry points give."""
import numpy as np
import pytest

from paper_2310_09204_amd import lib, meshes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [lib.FP64, lib.FP32_REFINE])
def test_device_mesh_and_solution_match_host_entry_points(ctx, precision):
    w = meshes.workload("square16", k=3)
    m = w.mesh
    print("case device io square16", precision, flush=True)
    dV, dT = lib.DeviceArray(np.asarray(m.vertices, dtype=np.float64)), lib.DeviceArray(np.asarray(m.triangles, dtype=np.int32))
    ph = lib.Problem(ctx, m.vertices, m.triangles, precision=precision)
    pd = lib.Problem(ctx, m.vertices, m.triangles, precision=precision, device_mesh=(dV.ptr, dT.ptr))
    assert np.array_equal(ph.matrix(), pd.matrix())
    Mh = lib.Preconditioner(ph, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                            factor_fp32=(precision == lib.FP32_REFINE))
    Md = lib.Preconditioner(pd, w.patch_of_triangle, w.coarse.vertices, w.coarse.triangles, w.coarse_of_triangle,
                            factor_fp32=(precision == lib.FP32_REFINE))
    phi_h, info_h, rc_h = ph.solve(g=w.g, precond=Mh, tol=1e-10, precision=precision)
    out = lib.DeviceArray(shape=(w.g.shape[0], pd.N))
    none, info_d, rc_d = pd.solve(g=w.g, precond=Md, tol=1e-10, precision=precision, device_out=out.ptr)
    assert none is None and rc_h == rc_d == 0
    assert np.array_equal(out.get(), phi_h)
    assert [i["iters"] for i in info_d] == [i["iters"] for i in info_h]
    for x in (Mh, Md, ph, pd, out, dV, dT):
        x.close()


def test_panel_assembly_returns_before_its_panels(ctx):
    # in panel mode bem_assemble returns with the panels queued: the caller's device mesh may go at
    # once (the call copied it), later calls queue behind the panels, and the phase times are NaN
    # until the panels have finished
    m = meshes.crossed(24)
    print("case early return panels crossed24", flush=True)
    dV, dT = lib.DeviceArray(np.asarray(m.vertices, dtype=np.float64)), lib.DeviceArray(np.asarray(m.triangles, dtype=np.int32))
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=4, device_mesh=(dV.ptr, dT.ptr), pair_panel_rows=512,
                    keep_order=True)
    dV.close()
    dT.close()
    t0 = p.info
    assert all(np.isnan(t0[k]) or t0[k] > 0 for k in ("t_far_s", "t_near_s", "t_contract_s"))
    assert t0["n_pair_panels"] > 1
    W = p.matrix()
    ref = lib.Problem(ctx, m.vertices, m.triangles, near_order=4, pair_panel_rows=512, keep_order=True)
    ctx.synchronize()
    assert np.array_equal(W, ref.matrix())
    i1 = p.info
    assert i1["t_far_s"] > 0 and i1["t_near_s"] > 0 and i1["t_contract_s"] > 0
    x = np.random.default_rng(4).standard_normal((3, p.N))
    assert np.array_equal(p.matvec(x), ref.matvec(x))
    p.close()
    ref.close()


def test_assembly_returns_before_its_contraction(ctx):
    # bem_assemble may return while the contraction into W still runs: the copy calls wait for it,
    # later calls queue behind it, and its device time is reported once it has finished
    m = meshes.crossed(24)
    print("case early return crossed24", flush=True)
    dV, dT = lib.DeviceArray(np.asarray(m.vertices, dtype=np.float64)), lib.DeviceArray(np.asarray(m.triangles, dtype=np.int32))
    p = lib.Problem(ctx, m.vertices, m.triangles, near_order=4, device_mesh=(dV.ptr, dT.ptr))
    dV.close()   # the device copy of the mesh may go as soon as the call has returned
    dT.close()
    t0 = p.info["t_contract_s"]
    assert np.isnan(t0) or t0 > 0
    W = p.matrix()
    ref = lib.Problem(ctx, m.vertices, m.triangles, near_order=4)
    ctx.synchronize()
    assert np.array_equal(W, ref.matrix())
    assert p.info["t_contract_s"] > 0 and ref.info["t_contract_s"] > 0
    x = np.random.default_rng(2).standard_normal((3, p.N))
    assert np.array_equal(p.matvec(x), ref.matvec(x))
    p.close()
    ref.close()
