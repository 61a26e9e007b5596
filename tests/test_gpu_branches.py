"""GPU parity on the correction-clamp and vanishing-gradient branches, with
the inputs of tests/test_oracle_branches.py (which pin the oracle there):
the HIP path against the oracle face by face at the plain bound, and against
the closed forms the pins use."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.common import gpu_run, vphase_tolerance

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


def test_uniform_alpha_clamped_and_homogeneous(vof, ctx, oracle_mod):
    """alpha = 0.37 under the deformation field on 16^3: every cell of the
    vanishing-gradient class, clamped faces present; classes, flags and every
    face's V_alpha equal the oracle's at the plain bound, alpha to 1e-13."""
    w = W.uniform_alpha(W.deform3d(16, steps=1), 0.37)
    print("[uniform-16] one step", flush=True)
    g = gpu_run(vof, ctx, w, steps=1)
    o = oracle_mod.Oracle(w.mesh)
    V, _, S, _ = o.geometry()
    Up = o.set_velocity(w.U0c, w.F0)
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    st = g["stats"]
    print(f"[uniform-16] fallback cells {st['fallback_cells']} clamped faces "
          f"{st['unreached_faces']}", flush=True)
    assert st["fallback_cells"] == w.mesh.n_cells
    assert st["unreached_faces"] == int((r["status"] == 1).sum()) > 0
    assert np.array_equal(g["cls"], r["rec"]["cls"])
    assert np.array_equal(g["status"], r["status"].astype(np.uint8))
    assert np.array_equal(g["kind"], r["kind"].astype(np.uint8))
    sdt = w.dt[0] * w.scale[0]
    tol = vphase_tolerance(w, V, sdt, S, Up)
    err = np.abs(g["vphase"] - r["vphase"])
    assert np.isfinite(g["vphase"]).all()
    assert (err <= tol).all(), (err / tol).max()
    assert np.abs(g["alpha"] - r["alpha"]).max() < 1e-13
    g["mesh"].close()


def test_isolated_cell_closed_form(vof, ctx):
    w = W.isolated_cell(8, 0.25, 0.5)
    g = gpu_run(vof, ctx, w, steps=1)
    c = w.meta["cell"]
    assert g["cls"][c] == 3 and g["stats"]["fallback_cells"] == 1
    frac = 0.25 * w.dt[0] * 8
    expect = np.zeros(w.mesh.n_cells)
    expect[c] = 0.5 * (1 - frac)
    expect[c + 1] = 0.5 * frac
    assert np.abs(g["alpha"] - expect).max() < 1e-15
    g["mesh"].close()


@pytest.mark.parametrize("k,status,lam", [(20.0, 0, 20.0), (31.0, 0, 31.0), (33.0, 1, 1.0),
                                          (40.0, 1, 1.0)])
def test_correction_branch_end(vof, ctx, oracle_mod, k, status, lam):
    w = W.scaled_translation(8, k)
    g = gpu_run(vof, ctx, w, steps=1)
    o = oracle_mod.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    flux = w.F0 != 0
    assert np.array_equal(g["status"], r["status"].astype(np.uint8))
    assert np.abs(g["lam"][flux] - r["lam"][flux]).max() <= 1e-12 * lam
    T = np.abs(w.F0) * w.dt[0]
    assert np.abs(g["vphase"] - r["vphase"]).max() <= 1e-13 * T.max()
    assert np.abs(g["alpha"] - r["alpha"]).max() < 1e-13
    g["mesh"].close()


@pytest.mark.parametrize("k,zero_u", [(40.0, False), (1.0, True)])
def test_unreachable_targets_take_the_donor_cell(vof, ctx, oracle_mod, k, zero_u):
    """Every face clamped (fluxes beyond the branch end, or no point velocity
    at all) on a random alpha field: V_alpha and alpha bitwise the oracle's
    (one product per face, the donor cell's alpha times F dt)."""
    w = W.scaled_translation(8, k)
    if zero_u:
        w.U0c[:] = 0.0
    w.alpha0 = np.random.default_rng(5).uniform(0.05, 0.95, w.mesh.n_cells)
    g = gpu_run(vof, ctx, w, steps=1)
    o = oracle_mod.Oracle(w.mesh)
    o.set_velocity(w.U0c, w.F0)
    r = o.step(w.alpha0, w.dt[0], w.scale[0])
    flux = w.F0 != 0
    assert (g["status"][flux] == 1).all() and (g["kind"][flux] == 4).all()
    assert g["stats"]["unreached_faces"] == int(flux.sum())
    assert np.array_equal(g["vphase"], r["vphase"])
    assert np.abs(g["alpha"] - r["alpha"]).max() <= 1e-15
    g["mesh"].close()
