"""The batched form: many meshes advanced by the same launches.

Every mesh's alpha, lambda and V_alpha after a batched run are bitwise those
of its own plain run with the same schedule (the batch kernels run the plain
kernels' code on each mesh's work, in the same order within each mesh), with
all three face kinds (tetrahedra, hexahedra, 2:1-refined hexahedra with
faces of up to eight points) in one batch; sampled meshes also match the
oracle.  Results do not depend on the launch configuration."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.common import oracle_run

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


def _instances(steps):
    ws = W.batch_instances(10, seed=7, n_range=(6, 14), steps=steps)
    ws += [W.rotate_tets(6, steps=steps, sample=4),
           W.rotate_tets(5, steps=steps, sample=4, centre=(0.5, 0.6, 0.5))]
    ws.append(W.uniform_alpha(W.deform3d(8, steps=steps), 0.0))  # nothing to clip
    return ws


def _upload(vof, ctx, ws):
    meshes = []
    for w in ws:
        m = vof.upload_mesh(ctx, w.mesh)
        vof.vof_set_alpha(m, w.alpha0)
        vof.vof_set_velocity(m, w.U0c, w.F0)
        meshes.append(m)
    return meshes


def _state(vof, m):
    return (vof.vof_read_alpha(m), vof.vof_read_face(m, vof.VOF_FACE_LAMBDA),
            vof.vof_read_face(m, vof.VOF_FACE_VPHASE), vof.vof_read_face(m, vof.VOF_FACE_STATUS))


def _schedule(ws, a, b):
    return (np.stack([w.dt[a:b] for w in ws]), np.stack([w.scale[a:b] for w in ws]))


def test_batch_equals_plain_runs(vof, ctx, oracle_mod):
    K1, K2 = 4, 3
    ws = _instances(K1 + K2)
    print(f"[batch] {len(ws)} meshes, cells {[w.mesh.n_cells for w in ws]}", flush=True)
    meshes = _upload(vof, ctx, ws)
    b = vof.vof_batch_create(ctx, meshes)
    # two calls in a row, the second under another launch configuration
    vof.vof_batch_advect(b, *_schedule(ws, 0, K1))
    c = vof.vof_batch_get_config(b)
    c.grid_flux, c.grid_clip, c.clip_claim, c.grid_plane, c.grid_cells = 64, 37, 1, 5, 11
    vof.vof_batch_set_config(b, c)
    vof.vof_batch_advect(b, *_schedule(ws, K1, K1 + K2))
    vof.vof_batch_synchronize(b)
    got = [_state(vof, m) for m in meshes]
    stats = [vof.vof_get_stats(m) for m in meshes]
    assert sum(s["geometric_faces"] for s in stats) > 0
    for w, m, st in zip(ws, meshes, stats):
        assert st["steps"] == K1 + K2
        assert st["face_fluxes"] == (K1 + K2) * int(np.count_nonzero(w.F0))
    # the same meshes, each alone
    for i, (w, m) in enumerate(zip(ws, meshes)):
        vof.vof_set_alpha(m, w.alpha0)
        vof.vof_advect(m, w.dt[:K1 + K2], w.scale[:K1 + K2])
        ref = _state(vof, m)
        for x, y in zip(ref, got[i]):
            assert np.array_equal(x, y), f"mesh {i} ({w.name}) differs from its plain run"
        st = vof.vof_get_stats(m)
        for k in ("geometric_faces", "interface_cells", "clip_pairs", "unreached_faces",
                  "correction_iters"):
            assert st[k] == stats[i][k], (i, k)
        assert st["ledger"] == stats[i]["ledger"]
    # sampled meshes against the oracle: a refined hex and a tet mesh
    for i in (1, 10):
        w = ws[i]
        _, a, _, _, _ = oracle_run(oracle_mod, w)
        assert np.abs(got[i][0] - a).max() < 1e-10, w.name
    b.close()
    for m in meshes:
        m.close()


def test_batch_refuses_bad_input(vof, ctx):
    ws = W.batch_instances(2, seed=3, n_range=(6, 8), steps=2)
    meshes = _upload(vof, ctx, ws)
    with pytest.raises(vof.VofError):
        vof.vof_batch_create(ctx, [meshes[0], meshes[0]])
    with pytest.raises(vof.VofError):
        vof.vof_batch_create(ctx, [])
    b = vof.vof_batch_create(ctx, meshes)
    dt, sc = _schedule(ws, 0, 2)
    dt[1, 1] = -1.0
    with pytest.raises(vof.VofError):
        vof.vof_batch_advect(b, dt, sc)
    p = vof.vof_get_params(meshes[0])
    p.narrow_band, p.wisps = 1, 1
    vof.vof_set_params(meshes[0], p)
    with pytest.raises(vof.VofError):
        vof.vof_batch_advect(b, *_schedule(ws, 0, 2))
    b.close()
    for m in meshes:
        m.close()


def test_autotune_advances_like_advect(vof, ctx, tmp_path):
    """vof_autotune advances the batch exactly as vof_batch_advect (one
    candidate configuration per step), keeps the fastest, and caches it under
    the GPU target and the batch's size bucket; a second batch of the same
    bucket takes the cached configuration."""
    import json
    K = 5
    ws = W.batch_instances(6, seed=11, n_range=(6, 12), steps=2 * K)
    meshes = _upload(vof, ctx, ws)
    b = vof.vof_batch_create(ctx, meshes)
    cache = str(tmp_path / "tune.json")
    c1 = vof.vof_autotune(b, *_schedule(ws, 0, K), cache_path=cache)
    assert c1 == vof.vof_batch_get_config(b).as_dict()
    vof.vof_batch_advect(b, *_schedule(ws, K, 2 * K))
    vof.vof_batch_synchronize(b)
    got = [vof.vof_read_alpha(m) for m in meshes]
    entries = json.load(open(cache))
    assert len(entries) == 1
    key, val = next(iter(entries.items()))
    assert key.startswith("gfx") and val == c1
    b.close()
    for w, m, a in zip(ws, meshes, got):
        vof.vof_set_alpha(m, w.alpha0)
        vof.vof_advect(m, w.dt[:2 * K], w.scale[:2 * K])
        assert np.array_equal(vof.vof_read_alpha(m), a)
    # the same bucket again: the cached entry, the same steps
    for w, m in zip(ws, meshes):
        vof.vof_set_alpha(m, w.alpha0)
    b2 = vof.vof_batch_create(ctx, meshes)
    c2 = vof.vof_autotune(b2, *_schedule(ws, 0, K), cache_path=cache)
    assert c2 == c1
    b2.close()
    for m in meshes:
        m.close()
