"""The served form: jobs of different meshes, sizes and lengths submitted to
a server with a fixed HBM budget, admitted as their state fits, stepped
together while resident.  Every job's alpha is bitwise that of the same
inputs advected alone (vof_advect), whatever else ran beside it; the budget
is never exceeded; a job larger than the budget is refused."""
from __future__ import annotations

import threading
import time

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


@pytest.fixture(scope="module")
def ctx(vof):
    c = vof.vof_context_create(0)
    yield c
    vof.vof_context_destroy(c)


def _templates(vof, ctx):
    tpls = [W.deformation_template("hex", 10), W.deformation_template("hex", 14),
            W.deformation_template("tets", 6)]
    meshes = [vof.upload_mesh(ctx, t.mesh) for t in tpls]
    return tpls, meshes


def _requests(tpls, count, seed, k_range=(3, 12)):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        i = int(rng.integers(len(tpls)))
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        reqs.append((i, *W.served_request(tpls[i], rng, K)))
    return reqs


def _alone(vof, tpl, mesh, a0, dt, sc):
    vof.vof_set_alpha(mesh, a0)
    vof.vof_set_velocity(mesh, tpl.U0c, tpl.F0)
    vof.vof_advect(mesh, dt, sc)
    return vof.vof_read_alpha(mesh)


def test_jobs_in_the_mix_equal_jobs_alone(vof, ctx, oracle_mod):
    tpls, meshes = _templates(vof, ctx)
    reqs = _requests(tpls, 24, seed=9)
    srv = vof.vof_server_create(ctx, 1 << 30)
    jobs = []
    # submitted from another thread in bursts of eight, 5 ms apart, so that
    # jobs join while others are resident
    def submit():
        for k, (i, a0, dt, sc) in enumerate(reqs):
            jobs.append(vof.vof_server_submit(srv, meshes[i], a0, tpls[i].U0c, tpls[i].F0, dt, sc))
            if k % 8 == 7:
                time.sleep(0.005)
    th = threading.Thread(target=submit)
    th.start()
    th.join()
    got = [vof.vof_server_wait(j) for j in jobs]
    st = vof.vof_server_get_stats(srv)
    print(f"[server] {st}", flush=True)
    assert st["jobs_done"] == len(reqs) and st["max_resident"] > 1
    assert st["face_fluxes"] == sum(len(dt) * int(np.count_nonzero(tpls[i].F0))
                                    for i, _, dt, _ in reqs)
    srv.close()
    for (i, a0, dt, sc), (a, lat) in zip(reqs, got):
        assert lat > 0
        assert np.array_equal(a, _alone(vof, tpls[i], meshes[i], a0, dt, sc))
    # one job against the oracle
    i, a0, dt, sc = reqs[0]
    o = oracle_mod.Oracle(tpls[i].mesh)
    o.set_velocity(tpls[i].U0c, tpls[i].F0)
    a, _, _, _ = o.advect(a0, dt, sc)
    assert np.abs(a - got[0][0]).max() < 1e-10
    for m in meshes:
        m.close()


def test_budget_bounds_admission(vof, ctx):
    tpls, meshes = _templates(vof, ctx)
    reqs = _requests(tpls, 10, seed=4)
    # state of the largest job, and a budget that holds two of them
    srv0 = vof.vof_server_create(ctx, 1 << 20)
    i, a0, dt, sc = reqs[0]
    big = W.deformation_template("hex", 24)
    mbig = vof.upload_mesh(ctx, big.mesh)
    a_big, dt_big, sc_big = W.served_request(big, np.random.default_rng(1), 4)
    with pytest.raises(vof.VofError) as e:
        vof.vof_server_submit(srv0, mbig, a_big, big.U0c, big.F0, dt_big, sc_big)
    assert e.value.code == vof.VOF_EBUSY
    srv0.close()
    budget = 6_000_000  # two or three of these jobs' states at a time
    srv = vof.vof_server_create(ctx, budget)
    jobs = [vof.vof_server_submit(srv, meshes[i], a0, tpls[i].U0c, tpls[i].F0, dt, sc)
            for i, a0, dt, sc in reqs]
    got = [vof.vof_server_wait(j)[0] for j in jobs]
    st = vof.vof_server_get_stats(srv)
    print(f"[server] budget {budget}: {st}", flush=True)
    assert st["peak_bytes"] <= budget and st["jobs_done"] == len(reqs)
    assert 1 <= st["max_resident"] < len(reqs)
    srv.close()
    for (i, a0, dt, sc), a in zip(reqs, got):
        assert np.array_equal(a, _alone(vof, tpls[i], meshes[i], a0, dt, sc))
    for m in meshes + [mbig]:
        m.close()
