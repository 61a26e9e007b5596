"""vof_advect_noalloc (for callers that cannot allocate device memory) against
vof_advect: two calls in a row on fresh copies of a mesh, the second on a
smaller mesh with fewer steps; alpha, lambda and V_alpha bitwise equal (the
same kernels, only the schedule's staging differs), and a schedule beyond the
staging maximum refused."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vof():
    import torch
    assert torch.cuda.is_available()
    import paper_1305_3417_amd as vof
    vof.lib()
    return vof


def _run(vof, ctx, w, n, noalloc):
    m = vof.upload_mesh(ctx, w.mesh)
    vof.vof_set_alpha(m, w.alpha0)
    vof.vof_set_velocity(m, w.U0c, w.F0)
    fn = vof.vof_advect_noalloc if noalloc else vof.vof_advect
    fn(m, w.dt[:n], w.scale[:n])
    out = (vof.vof_read_alpha(m), vof.vof_read_face(m, vof.VOF_FACE_LAMBDA),
           vof.vof_read_face(m, vof.VOF_FACE_VPHASE), vof.vof_get_stats(m))
    m.close()
    return out


def test_noalloc_matches_advect(vof):
    ctx = vof.vof_context_create(0)
    for w, n in ((W.deform3d(16, steps=6), 6), (W.rotate_tets(8, steps=3, sample=4), 3)):
        print(f"[noalloc] {w.name} cells {w.mesh.n_cells} steps {n}", flush=True)
        ref = _run(vof, ctx, w, n, noalloc=False)
        got = _run(vof, ctx, w, n, noalloc=True)
        for x, y in zip(ref[:3], got[:3]):
            assert np.array_equal(x, y)
        assert got[3]["steps"] == n and got[3]["face_fluxes"] == ref[3]["face_fluxes"]
    vof.vof_context_destroy(ctx)


def test_noalloc_refuses_long_schedule(vof):
    ctx = vof.vof_context_create(0)
    w = W.deform3d(8, steps=1)
    m = vof.upload_mesh(ctx, w.mesh)
    vof.vof_set_alpha(m, w.alpha0)
    vof.vof_set_velocity(m, w.U0c, w.F0)
    n = vof.VOF_NOALLOC_MAX_STEPS + 1
    with pytest.raises(vof.VofError) as e:
        vof.vof_advect_noalloc(m, np.full(n, w.dt[0]), np.ones(n))
    assert e.value.code == vof.VOF_EINVAL
    assert np.array_equal(vof.vof_read_alpha(m), w.alpha0)
    m.close()
    vof.vof_context_destroy(ctx)
