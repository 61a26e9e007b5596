"""GPU parity: the HIP path against the CPU oracle on identical seeded inputs.

Tolerances (FP64 on both sides, different summation orders and different
geometric routes).  G_f = |S_f| max_i |s dt U_p_i| is the gross swept volume
of face f: the flux polyhedron volume is a signed sum of terms of that size,
so any FP64 evaluation of it is accurate to a few eps * G_f, however small
the net flux F_f dt.
  lambda_f            the oracle's own volume at lam_gpu within the V_alpha
                      bound below of F_f dt (lambda itself is ill-conditioned
                      where V' is small; relative 1e-8 sanity)
  V_{f,alpha}         1e-12 * max(|F_f| dt, G_f, 1e-2 max(V_owner, d_f^3)) per
                      face, d_f the face's diameter; the floor is the FP64
                      rounding of tetrahedra whose edges are as long as the
                      face (about 20 eps h^3 on hex faces) when flux and sweep
                      are tiny
  plane normal        1e-12 (components; same classes required)
  alpha after N steps 1e-10 absolute
  conservation        sum V alpha + ledger within 1e-12 relative
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.common import gpu_run, oracle_run, vphase_tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vof():
    import torch
    assert torch.cuda.is_available()
    import paper_1305_3417_amd as vof
    vof.lib()
    return vof


@pytest.fixture(scope="module")
def ctx(vof):
    c = vof.vof_context_create(0)
    yield c
    vof.vof_context_destroy(c)


def _compare_step(vof, ctx, oracle_mod, w, alpha=None, label="", gradient="nag"):
    """One step from `alpha`: planes, lambda, V_alpha and alpha."""
    a0 = w.alpha0 if alpha is None else alpha
    print(f"[{label}] one step, cells {w.mesh.n_cells} faces {w.mesh.n_faces}", flush=True)
    params = {"gradient": vof.VOF_GRADIENT_LSQ} if gradient == "lsq" else None
    g = gpu_run(vof, ctx, w, steps=1, alpha=a0, params=params)
    o = oracle_mod.Oracle(w.mesh, gradient=gradient)
    V, _, S, _ = o.geometry()
    Up = o.set_velocity(w.U0c, w.F0)
    r = o.step(a0, w.dt[0], w.scale[0])
    sdt = w.scale[0] * w.dt[0]
    rec = r["rec"]
    assert np.array_equal(g["cls"], rec["cls"]), "cell classes differ"
    iface = rec["cls"] == 1
    assert np.abs(g["n"][iface] - rec["n"][iface]).max(initial=0) < 1e-12
    flux = w.F0 != 0
    assert np.array_equal(g["status"], r["status"].astype(np.uint8)), "correction flags differ"
    rel = np.abs(g["lam"][flux] - r["lam"][flux]) / np.maximum(np.abs(r["lam"][flux]), 1e-300)
    ok = g["status"][flux] == 0
    assert rel[ok].max(initial=0) < 1e-8
    # clamped faces: lambda at the extremum of V, located from a cubic fit
    assert rel[~ok].max(initial=0) < 1e-9
    # the oracle's own volume at the GPU's lambda (sampled)
    tol = vphase_tolerance(w, V, sdt, S, Up)
    fl = np.flatnonzero(flux)
    for f in fl[:: max(1, fl.size // 400)]:
        if g["status"][f] == 0:
            res = abs(o.flux_volume(f, w.dt[0], w.scale[0], g["lam"][f]) - w.F0[f] * sdt)
            assert res <= tol[f]
    assert np.array_equal(g["kind"], r["kind"].astype(np.uint8))
    err = np.abs(g["vphase"] - r["vphase"])
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, f"{bad.size} faces beyond tolerance, worst {(err / tol).max():.3g}x"
    assert np.abs(g["alpha"] - r["alpha"]).max() < 1e-13
    g["mesh"].close()
    return g, r


def test_disc2d_one_step(vof, ctx, oracle_mod):
    w = W.disc2d()
    _compare_step(vof, ctx, oracle_mod, w, label="disc2d")


def test_disc2d_full_run(vof, ctx, oracle_mod):
    """All 50 steps: alpha within 1e-10, conservation and boundedness."""
    w = W.disc2d()
    g = gpu_run(vof, ctx, w)
    o, a, st, lam, vp = oracle_run(oracle_mod, w)
    V, _, _, _ = o.geometry()
    assert np.abs(g["alpha"] - a).max() < 1e-10
    m0 = (w.alpha0 * V).sum()
    gs = g["stats"]
    assert abs(gs["mass"] + gs["ledger"] - m0) <= 1e-12 * m0
    assert gs["alpha_min"] > -1e-12 and gs["alpha_max"] < 1 + 1e-12
    assert gs["capacity_overflows"] == 0 and gs["unreached_faces"] == 0
    assert gs["face_fluxes"] == 50 * int((w.F0 != 0).sum())
    g["mesh"].close()


def test_slab_translation_exact(vof, ctx):
    w = W.translate_slab(16, 2, a=0.3, b=0.55, U=(0.25, 0.0, 0.0), steps=24)
    g = gpu_run(vof, ctx, w)
    assert np.abs(g["alpha"] - W.slab_exact(w, 24)).max() < 1e-13
    g["mesh"].close()


def test_translation_is_exact_prism(vof, ctx):
    """Uniform translation: lam = 1 to round-off, no correction iterations."""
    w = W.disc2d(steps=1)
    g = gpu_run(vof, ctx, w, steps=1)
    flux = w.F0 != 0
    assert np.abs(g["lam"][flux] - 1.0).max() < 1e-13
    assert g["iters"][flux].max() <= 1
    g["mesh"].close()


def test_deform3d_small_steps(vof, ctx, oracle_mod):
    w = W.deform3d(24, steps=8)
    _compare_step(vof, ctx, oracle_mod, w, label="deform3d-24")
    g = gpu_run(vof, ctx, w)
    o, a, st, lam, vp = oracle_run(oracle_mod, w)
    assert np.abs(g["alpha"] - a).max() < 1e-10
    V, _, S, _ = o.geometry()
    Up = o.set_velocity(w.U0c, w.F0)
    tol = vphase_tolerance(w, V, w.scale[-1] * w.dt[-1], S, Up)
    assert (np.abs(g["vphase"] - vp) <= tol).all()
    g["mesh"].close()


def test_rotate_tets_small(vof, ctx, oracle_mod):
    w = W.rotate_tets(10, steps=6, sample=8)
    _compare_step(vof, ctx, oracle_mod, w, label="tets-10")
    g = gpu_run(vof, ctx, w)
    o, a, st, lam, vp = oracle_run(oracle_mod, w)
    assert np.abs(g["alpha"] - a).max() < 1e-10
    gs = g["stats"]
    print(f"[tets-10] alpha range [{gs['alpha_min']:.3e}, {gs['alpha_max']:.3e}], "
          f"{gs['unreached_faces']} clamped faces in {w.n_steps} steps", flush=True)
    # cell Courant 0.5 (the oracle's alpha stays in [0, 0.9959] here)
    assert gs["alpha_min"] >= -1e-12 and gs["alpha_max"] <= 1 + 1e-12
    g["mesh"].close()


def test_rotate_tets_stencil_complete(vof, ctx, oracle_mod):
    """A slotted sphere whose orbit stays four cells from the walls: every flux
    polyhedron of a geometric face lies inside its stencil (the point-cells
    of its points), on both sides, over several steps."""
    w = W.rotate_tets(20, steps=4, sample=6, centre=(0.5, 0.65, 0.5))
    g = gpu_run(vof, ctx, w, params={"check_stencil": 1})
    o, a, st, lam, vp = oracle_run(oracle_mod, w, check_leak=True)
    assert st["max_leak"] < 1e-12
    assert g["stats"]["stencil_leaks"] == 0
    err = np.abs(g["alpha"] - a)
    bad = np.flatnonzero(err >= 1e-10)
    assert bad.size == 0, (bad[:10], g["alpha"][bad[:10]], a[bad[:10]], g["stats"])
    g["mesh"].close()


def test_rerun_is_bitwise_identical(vof, ctx):
    """Every reduction has a fixed order and no result goes through a race:
    the same run three times gives bit-identical fields, also with the
    stencil check (every flux tet through the general clipper, where the
    rare pairs of five or more planes share one polytope per wavefront), with
    the least-squares gradient on tetrahedra (cells of about 70 neighbours,
    spread over the lanes of the cell's group), and on a refined mesh (cells
    of up to 15 faces whose interface cells are evaluated by half or whole
    waves, paired in the order of a list filled by atomics)."""
    tets = W.rotate_tets(20, steps=4, sample=6, centre=(0.5, 0.65, 0.5))
    refined = W.deform3d_refined(16, steps=12)
    lsq = {"gradient": vof.VOF_GRADIENT_LSQ}
    for w, params in ((tets, {"check_stencil": 0}), (tets, {"check_stencil": 1}),
                      (tets, lsq), (refined, {}), (refined, lsq)):
        ref = None
        for _ in range(3):
            g = gpu_run(vof, ctx, w, params=params)
            cur = (g["alpha"].copy(), g["vphase"].copy(), g["lam"].copy())
            assert g["stats"]["capacity_overflows"] == 0
            g["mesh"].close()
            if ref is None:
                ref = cur
            else:
                for x, y in zip(ref, cur):
                    assert np.array_equal(x, y)


def test_set_alpha_restarts_the_run(vof, ctx):
    """Positioning starts from each cell's stored plane; vof_set_alpha clears
    the planes, so the same run on the same mesh after it is bitwise the
    first, and a reconstruction from stored planes agrees to the positioning
    tolerance with one from cleared planes."""
    w = W.deform3d(16, steps=8)
    m = vof.upload_mesh(ctx, w.mesh)
    vof.vof_set_velocity(m, w.U0c, w.F0)
    runs = []
    for _ in range(2):
        vof.vof_set_alpha(m, w.alpha0)
        vof.vof_advect(m, w.dt, w.scale)
        runs.append((vof.vof_read_alpha(m), vof.vof_read_face(m, vof.VOF_FACE_VPHASE)))
    for x, y in zip(*runs):
        assert np.array_equal(x, y)
    # the planes of alpha after the run: from the stored planes, and from cleared ones
    vof.vof_reconstruct(m)
    cls1, n1, s1 = vof.vof_read_planes(m)
    a = vof.vof_read_alpha(m)
    vof.vof_set_alpha(m, a)
    vof.vof_reconstruct(m)
    cls2, n2, s2 = vof.vof_read_planes(m)
    assert np.array_equal(cls1, cls2)
    iface = cls1 == 1
    assert iface.any()
    # the normals do not depend on the planes (outside the interface cells the
    # stored planes are those of earlier steps, or cleared)
    assert np.array_equal(n1[iface], n2[iface])
    # both meet the fill level to 1e-15 of the cell volume; a plane cutting a
    # corner of alpha ~ 1e-10 moves by ~3e-9 h for that (dV/ds ~ (6V)^(2/3) / 2)
    assert np.abs(s1[iface] - s2[iface]).max() <= 1e-8 / 16
    m.close()


def test_step_graph_replays_match_eager(vof, ctx):
    """Steps replayed from the captured graph (profiling off; the plane kernel
    on a side stream) against the same steps launched kernel by kernel on one
    stream (profiling on): bitwise equal after every call, with eager work
    (reads, a reconstruction, parameter changes that force new captures: the
    stencil check, the narrow band with wisps, the LSQ gradient) between the
    replays."""
    w = W.deform3d(16, steps=16)
    meshes = []
    for prof in (False, True):
        m = vof.upload_mesh(ctx, w.mesh)
        vof.vof_set_alpha(m, w.alpha0)
        vof.vof_set_velocity(m, w.U0c, w.F0)
        vof.vof_profile_enable(m, prof)
        meshes.append(m)

    def state(m):
        return (vof.vof_read_alpha(m), vof.vof_read_face(m, vof.VOF_FACE_LAMBDA),
                vof.vof_read_face(m, vof.VOF_FACE_VPHASE))

    def same():
        for x, y in zip(state(meshes[0]), state(meshes[1])):
            assert np.array_equal(x, y)

    k = 0
    for n, params in [(3, None), (1, None), (2, {"check_stencil": 1}), (2, {"check_stencil": 0}),
                      (2, {"narrow_band": 1, "wisps": 1}), (2, {"gradient": vof.VOF_GRADIENT_LSQ}),
                      (4, {"narrow_band": 0, "wisps": 0, "gradient": vof.VOF_GRADIENT_NAG})]:
        for m in meshes:
            if params:
                p = vof.vof_get_params(m)
                for key, v in params.items():
                    setattr(p, key, v)
                vof.vof_set_params(m, p)
            vof.vof_advect(m, w.dt[k:k + n], w.scale[k:k + n])
        k += n
        same()
        for m in meshes:
            vof.vof_reconstruct(m)
        assert all(np.array_equal(x, y) for x, y in
                   zip(vof.vof_read_planes(meshes[0]), vof.vof_read_planes(meshes[1])))
    for m in meshes:
        m.close()


def test_shear_adaptive_courant(vof, ctx, oracle_mod):
    """The shear field (eq. 4.5) with the adaptive Courant time step through
    the same kernels, 16^3 to T = 3 (71 steps, through the reversal): one step
    at t = 0 and one from the oracle's state at mid-run (the longest steps),
    then alpha and the advection error E_g after the whole run."""
    import dataclasses
    w = W.shear3d(16)
    _compare_step(vof, ctx, oracle_mod, w, label="shear-16")
    mid = w.n_steps // 2
    o, a_mid, st, lam, vp = oracle_run(oracle_mod, w, steps=mid)
    wm = dataclasses.replace(w, dt=w.dt[mid:], scale=w.scale[mid:])
    _compare_step(vof, ctx, oracle_mod, wm, alpha=a_mid, label="shear-16-mid")
    g = gpu_run(vof, ctx, w)
    o, a, st, lam, vp = oracle_run(oracle_mod, w)
    assert np.abs(g["alpha"] - a).max() < 1e-10
    V = o.geometry()[0]
    eg_gpu = float((V * np.abs(g["alpha"] - w.alpha0)).sum())
    eg_orc = float((V * np.abs(a - w.alpha0)).sum())
    print(f"[shear-16] E_g gpu {eg_gpu:.6e} oracle {eg_orc:.6e}", flush=True)
    assert abs(eg_gpu - eg_orc) <= 1e-10 * eg_orc
    g["mesh"].close()


@pytest.mark.parametrize("case", ["deform3d", "tets"])
def test_lsq_gradient_reconstruction(vof, ctx, oracle_mod, case):
    """The generalized least-squares gradient (Section 2.2.1) in place of NAG:
    one step at step level (classes, normals to 1e-12, lambda, V_alpha), then
    alpha after several steps."""
    w = W.deform3d(16, steps=6) if case == "deform3d" else W.rotate_tets(10, steps=6, sample=8)
    _compare_step(vof, ctx, oracle_mod, w, label=f"lsq-{case}", gradient="lsq")
    g = gpu_run(vof, ctx, w, params={"gradient": vof.VOF_GRADIENT_LSQ})
    o, a, st, lam, vp = oracle_run(oracle_mod, w, gradient="lsq")
    assert np.abs(g["alpha"] - a).max() < 1e-10
    g["mesh"].close()


def test_narrow_band_leaves_bulk_cells(vof, ctx, oracle_mod):
    """Narrow band (Section 2.3), one step of the deformation field: the bulk
    cells (every cell sharing a point exactly 0, or all exactly 1) keep their
    alpha bit for bit; the others match the oracle's band step."""
    w = W.deform3d(24, steps=2)
    o = oracle_mod.Oracle(w.mesh, band=True)
    o.set_velocity(w.U0c, w.F0)
    bulk = o.bulk_cells(w.alpha0)
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    g = gpu_run(vof, ctx, w, steps=1, params={"narrow_band": 1})
    assert np.array_equal(g["alpha"][bulk], w.alpha0[bulk])
    assert np.abs(g["alpha"] - r["alpha"]).max() < 1e-13
    g["mesh"].close()


WISP_CASES = {
    "deform3d": lambda: W.deform3d(24, steps=40),
    "deform3d-128": lambda: W.deform3d(128, steps=6),
    "tets": lambda: W.rotate_tets(10, steps=12, sample=8),
    "shear": lambda: W.shear3d(16, steps=30),
    "disc2d": lambda: W.disc2d(),
}


@pytest.mark.parametrize("case", sorted(WISP_CASES))
def test_narrow_band_and_wisps(vof, ctx, oracle_mod, case):
    """Narrow band and wisp redistribution (Section 2.3) over a run: alpha
    within 1e-10 of the oracle's, volume conserved with the ledger, and a
    second run bitwise identical (the wisp and receiver lists are filled by
    atomics in any order, every sum runs in stencil order)."""
    w = WISP_CASES[case]()
    params = {"narrow_band": 1, "wisps": 1}
    print(f"[wisps-{case}] cells {w.mesh.n_cells} steps {w.n_steps}", flush=True)
    g = gpu_run(vof, ctx, w, params=params)
    o, a, st, lam, vp = oracle_run(oracle_mod, w, band=True, wisps=True)
    V = o.geometry()[0]
    gs = g["stats"]
    print(f"[wisps-{case}] wisps gpu {gs['wisps']} ({gs['wisps_left']} left) oracle "
          f"{st['n_wisps']} ({st['n_wisps_left']} left); alpha range gpu "
          f"[{gs['alpha_min']:.3e}, {gs['alpha_max']:.3e}] oracle [{a.min():.3e}, {a.max():.3e}]",
          flush=True)
    assert np.abs(g["alpha"] - a).max() < 1e-10
    m0 = (w.alpha0 * V).sum()
    assert abs(gs["mass"] + gs["ledger"] - m0) <= 1e-12 * m0
    assert gs["wisps"] > 0 and st["n_wisps"] > 0
    # the redistribution keeps alpha in [0, 1] (the plain update alone does
    # not: corrected polyhedra of neighbouring faces overlap where the sweep
    # varies along the face, e.g. -4e-3 on the 16^3 shear case)
    assert gs["alpha_min"] >= -1e-12 and gs["alpha_max"] <= 1 + 1e-12
    g2 = gpu_run(vof, ctx, w, params=params)
    assert np.array_equal(g2["alpha"], g["alpha"])
    g["mesh"].close()
    g2["mesh"].close()


def test_refined_mesh_advection(vof, ctx, oracle_mod):
    """A hex mesh refined once around the sphere (2:1, faces of 4-6 points,
    cells of up to 15 faces, coplanar faces of a coarse cell one clipping
    plane): one step compared quantity by quantity, then alpha after 8 steps
    with every flux polyhedron checked to stay inside its stencil."""
    w = W.deform3d_refined(12, steps=8)
    _compare_step(vof, ctx, oracle_mod, w, label="refined-12")
    g = gpu_run(vof, ctx, w, params={"check_stencil": 1})
    o, a, st, lam, vp = oracle_run(oracle_mod, w, check_leak=True)
    assert st["max_leak"] < 1e-12 and g["stats"]["stencil_leaks"] == 0
    assert np.abs(g["alpha"] - a).max() < 1e-10
    V = o.geometry()[0]
    m0 = (w.alpha0 * V).sum()
    assert abs(g["stats"]["mass"] + g["stats"]["ledger"] - m0) <= 1e-12 * m0
    g["mesh"].close()


def test_geometric_mapping(vof, ctx, oracle_mod):
    """Algorithm 2 (Section 3): the oracle's alpha after six deformation steps
    on 16^3 is mapped onto the mesh refined in its interface cells, on the GPU
    and by the oracle (each reconstructing the same alpha), then mapped back
    by union; host and device map arrays; a bad map is refused."""
    import torch
    from workloads.refine import refine_hex
    n = 16
    w0 = W.deform3d(n, steps=6)
    _, a_old, _, _, _ = oracle_run(oracle_mod, w0)
    m1, parent, (coff, cells) = refine_hex(n, (a_old > 1e-12) & (a_old < 1 - 1e-12))
    print(f"[mapping] {w0.mesh.n_cells} -> {m1.n_cells} cells", flush=True)
    o0, o1 = oracle_mod.Oracle(w0.mesh), oracle_mod.Oracle(m1)
    ident = np.arange(m1.n_cells + 1, dtype=np.int32)
    e1 = o1.map_alpha(o0, a_old, ident, parent)
    e0 = o0.map_alpha(o1, e1, coff, cells)
    src = vof.upload_mesh(ctx, w0.mesh)
    dst = vof.upload_mesh(ctx, m1)
    vof.vof_set_alpha(src, a_old)
    vof.vof_map_alpha(dst, src, ident, parent)
    g1 = vof.vof_read_alpha(dst)
    assert np.abs(g1 - e1).max() < 1e-11
    V0, V1 = o0.geometry()[0], o1.geometry()[0]
    assert abs((g1 * V1).sum() - (a_old * V0).sum()) <= 1e-13 * (a_old * V0).sum()
    # back to the uniform mesh, map arrays on the device
    back = vof.upload_mesh(ctx, w0.mesh)
    vof.vof_map_alpha(back, dst, torch.as_tensor(coff.astype(np.int32), device="cuda"),
                      torch.as_tensor(cells.astype(np.int32), device="cuda"))
    g0 = vof.vof_read_alpha(back)
    assert np.abs(g0 - e0).max() < 1e-11 and np.abs(g0 - a_old).max() < 1e-11
    bad = parent.copy()
    bad[3] = w0.mesh.n_cells
    with pytest.raises(vof.VofError):
        vof.vof_map_alpha(dst, src, ident, bad)
    with pytest.raises(vof.VofError):
        vof.vof_map_alpha(back, dst, torch.as_tensor(coff.astype(np.int32), device="cuda"),
                          torch.as_tensor(np.full(cells.size, -1, np.int32), device="cuda"))
    for h in (src, dst, back):
        h.close()


@pytest.mark.parametrize("gradient", ["nag", "lsq"])
def test_sphere_reconstruction_error(vof, ctx, oracle_mod, gradient):
    """Reconstruction alone (vof_reconstruct) of an exact sphere on 32^3
    hexahedra: classes equal, and the volume of symmetric difference E_vsd
    (Section 4.1) of the GPU's planes equals that of the oracle's planes."""
    from tests.reconstruction_error import vsd
    from workloads import fields
    c, r = np.array([0.5123, 0.4871, 0.5036]), 0.15
    m = W.hex_mesh(32, 32, 32)
    a0 = fields.ball_box_fraction(c, r, m.cell_lo, m.cell_hi)
    h = vof.upload_mesh(ctx, m)
    p = vof.vof_get_params(h)
    p.gradient = vof.VOF_GRADIENT_LSQ if gradient == "lsq" else vof.VOF_GRADIENT_NAG
    vof.vof_set_params(h, p)
    vof.vof_set_alpha(h, a0)
    vof.vof_reconstruct(h)
    cls, nrm, s = vof.vof_read_planes(h)
    h.close()
    rec = oracle_mod.Oracle(m, gradient=gradient).reconstruct(a0)
    assert np.array_equal(cls, rec["cls"])
    e_gpu = vsd(m, cls, nrm, s, (c, r))
    e_orc = vsd(m, rec["cls"], rec["n"], rec["s"], (c, r))
    print(f"[vsd-{gradient}] E_vsd gpu {e_gpu:.6e} oracle {e_orc:.6e}", flush=True)
    assert abs(e_gpu - e_orc) <= 1e-9 * e_orc


def test_empty_and_full_fields(vof, ctx):
    w = W.deform3d(12, steps=3)
    for val in (0.0, 1.0):
        g = gpu_run(vof, ctx, w, alpha=np.full(w.mesh.n_cells, val))
        assert np.abs(g["alpha"] - val).max() < 1e-13
        assert g["stats"]["geometric_faces"] == 0
        g["mesh"].close()


# (workload, first step): the later starts take the GPU's own state after
# that many steps (the interface stretched furthest, T/2, on the deformation
# case; a thousand steps into the rotation on the tets)
FULL_SIZE = {
    "deform3d-128": (lambda: W.deform3d(128, steps=1), 0),
    "deform3d-128-mid": (lambda: W.deform3d(128), 768),
    "shear3d-128": (lambda: W.shear3d(128, steps=1), 0),
    "tets-80": (lambda: W.rotate_tets(80, steps=1), 0),
    "tets-80-mid": (lambda: W.rotate_tets(80, steps=1001), 1000),
}


@pytest.mark.parametrize("case", sorted(FULL_SIZE))
def test_full_size_sampled(vof, ctx, oracle_mod, case):
    """The 128^3 deformation case (the benchmark's, in its launch
    configuration), the 128^3 shear case and the 80^3 x 6 jittered-tet case:
    one step from alpha^0, and for the deformation and tet cases one step
    from the GPU's state in the middle of the run, sampled faces and cells
    checked one by one against the oracle from the same state."""
    import dataclasses
    make, start = FULL_SIZE[case]
    w = make()
    if start:
        print(f"[{case}] gpu advances {start} steps", flush=True)
        g0 = gpu_run(vof, ctx, w, steps=start)
        a = g0["alpha"]
        g0["mesh"].close()
        w = dataclasses.replace(w, alpha0=a, dt=w.dt[start:start + 1],
                                scale=w.scale[start:start + 1])
    print(f"[{case}] gpu step", flush=True)
    g = gpu_run(vof, ctx, w, steps=1)
    rng = np.random.default_rng(17)
    geo = np.flatnonzero(g["kind"] == 3)
    flux = np.flatnonzero(w.F0 != 0)
    faces = np.unique(np.concatenate([rng.choice(geo, min(1500, geo.size), replace=False),
                                      rng.choice(flux, 1500, replace=False)]))
    # cells whose alpha is checked: interface cells and their faces
    icells = np.flatnonzero(g["cls"] == 1)
    cells = rng.choice(icells, min(300, icells.size), replace=False)
    m = w.mesh
    own, nei = m.owner, m.neighbour
    cell_faces = np.flatnonzero(np.isin(own, cells) |
                                np.isin(np.concatenate([nei, -np.ones(m.n_faces - m.n_internal,
                                                                      dtype=nei.dtype)]), cells))
    faces = np.unique(np.concatenate([faces, cell_faces]))
    print(f"[{case}] oracle on {faces.size} faces", flush=True)
    o = oracle_mod.Oracle(m)
    V, _, S, _ = o.geometry()
    Up = o.set_velocity(w.U0c, w.F0)
    sdt = w.scale[0] * w.dt[0]
    st_off, st_cells = o.stencil()
    need = np.unique(np.concatenate([st_cells[st_off[f]:st_off[f + 1]] for f in faces]))
    rec = o.reconstruct_subset(w.alpha0, need)
    assert np.array_equal(g["cls"][need], rec["cls"][need])
    iface = need[rec["cls"][need] == 1]
    assert np.abs(g["n"][iface] - rec["n"][iface]).max() < 1e-12
    r = o.faces_subset(w.dt[0], w.scale[0], w.alpha0, faces)
    assert np.array_equal(g["status"][faces], r["status"].astype(np.uint8))
    fl = (w.F0[faces] != 0) & (r["status"] == 0)
    rel = np.abs(g["lam"][faces][fl] - r["lam"][fl]) / np.abs(r["lam"][fl])
    # lambda to 1e-8, or to what a volume error within the V_alpha bound
    # moves it by (about tol / |F dt| relative where V is near-linear in
    # lambda): near the field's reversal (mid-run) the fluxes are tiny
    tol_all = vphase_tolerance(w, V, sdt, S, Up)
    lam_bound = np.maximum(1e-8, 10.0 * tol_all[faces][fl] / np.abs(w.F0[faces][fl] * sdt))
    assert (rel <= lam_bound).all(), (rel / lam_bound).max()
    # the oracle's own volume at the GPU's lambda meets F dt (lambda itself is
    # ill-conditioned where V' is small; the volume is what the update uses)
    for f in faces[fl][::3]:
        res = abs(o.flux_volume(f, w.dt[0], w.scale[0], g["lam"][f]) - w.F0[f] * sdt)
        assert res <= tol_all[f]
    ref = r["vphase"].copy()
    tol = tol_all[faces]
    clamp = int(((w.F0[faces] != 0) & (r["status"] == 1)).sum())
    print(f"[{case}] {clamp} sampled faces clamped at the extremum (donor cell)", flush=True)
    err = np.abs(g["vphase"][faces] - ref)
    assert (err <= tol).all(), (faces[err > tol][:5], (err / tol).max())
    # on the tet mesh, faces with more candidate cells than a group's share
    # take the chunked candidate path, so the checked step went through it
    resc = g["stats"]["chunk_rescans"]
    print(f"[{case}] {resc} chunk rescans", flush=True)
    if case.startswith("tets"):
        assert resc > 0
    # alpha of the sampled cells from the oracle's face volumes, to 1e-13 plus
    # the faces' own bounds over the cell volume
    vph = dict(zip(faces.tolist(), ref.tolist()))
    ftol = dict(zip(faces.tolist(), tol.tolist()))
    for c in cells[:100]:
        acc = 0.0
        bound = 1e-13
        for f in cell_faces:
            if own[f] == c:
                acc += vph[f]
                bound += ftol[f] / V[c]
            elif f < m.n_internal and nei[f] == c:
                acc -= vph[f]
                bound += ftol[f] / V[c]
        assert abs(g["alpha"][c] - (w.alpha0[c] - acc / V[c])) < bound
    g["mesh"].close()
