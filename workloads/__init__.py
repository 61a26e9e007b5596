"""Seeded synthetic workloads for the geometric PLIC VoF flux path.

A workload is a mesh plus everything the advection needs as input: the initial
volume fraction, the cell-centred reference velocity U0_c, the reference face
flux F0_f (discretely divergence free, eq. 2.4) and a time-step schedule in
which step n uses velocity scale[n] * U0 and flux scale[n] * F0 with step
length dt[n].  Both the oracle and the GPU library are fed the same arrays.

Workloads (sizes as in the paper's advection tests, Section 4.2):
  disc2d      64x64x1 hex layer, disc r=0.15 at (0.5, 0.75), U=(1, 0.5, 0),
              Co 0.5, 50 steps
  deform3d    N^3 hex (N=128 for the full case), sphere r=0.15 at
              (0.35, 0.35, 0.35), deformation field (eq. 4.6) with
              cos(pi t/T), T=3, Co 0.5 (dt = 1/(4N))
  rotate_tets jittered Kuhn tets on an N^3 lattice (N=80 full), slotted sphere
              r=0.15 at (0.5, 0.75, 0.5), slot width 0.05, rigid rotation about
              z through (0.5, 0.5) at 2 pi per unit time, cell Courant number
              at most 0.5
  shear3d     N^3 hex, sphere r=0.15 at (0.5, 0.75, 0.25), shear field (eq. 4.5)
              with cos(pi t/T), T=3, u_max=1, R=0.5, adaptive Courant time step
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields
from .meshes import Mesh, hex_mesh, kuhn_tet_mesh, single_cell_mesh  # noqa: F401


@dataclass
class Workload:
    name: str
    mesh: Mesh
    alpha0: np.ndarray      # (C,)
    U0c: np.ndarray         # (C, 3)
    F0: np.ndarray          # (F,)
    dt: np.ndarray          # (N,)
    scale: np.ndarray       # (N,)
    meta: dict = field(default_factory=dict)

    @property
    def n_steps(self) -> int:
        return int(self.dt.shape[0])


def disc2d(n: int = 64, steps: int = 50) -> Workload:
    """Disc r=0.15 at (0.5, 0.75) on an n x n x 1 layer, U = (1, 0.5, 0), Co 0.5."""
    h = 1.0 / n
    m = hex_mesh(n, n, 1, (0.0, 0.0, 0.0), (1.0, 1.0, h))
    a0 = fields.disc_square_fraction((0.5, 0.75), 0.15, m.cell_lo[:, :2], m.cell_hi[:, :2])
    U = np.array([1.0, 0.5, 0.0])
    Uc = np.broadcast_to(U, (m.n_cells, 3)).copy()
    F0 = fields.flux_constant(m, U)
    dt = 0.5 * h / np.sqrt(1.25)
    return Workload("disc2d", m, a0, Uc, F0, np.full(steps, dt), np.ones(steps),
                    meta={"n": n, "co": 0.5, "U": U.tolist()})


def deform3d(n: int = 128, steps: int | None = None, T: float = 3.0,
             centre=(0.35, 0.35, 0.35), radius: float = 0.15) -> Workload:
    """Sphere in the periodic deformation field (eq. 4.6), fixed dt = 1/(4n).

    max |U0| over mesh points is 2, so dt = 0.5 h / 2 gives Co 0.5.  Step n uses
    scale cos(pi (t_n + dt/2) / T).  The default step count reaches T.
    """
    m = hex_mesh(n, n, n)
    a0 = fields.ball_box_fraction(centre, radius, m.cell_lo, m.cell_hi)
    Uc = fields.deformation_velocity(m.cell_centroids())
    F0 = fields.flux_deformation(m)
    dt = 1.0 / (4 * n)
    N = int(round(T / dt)) if steps is None else steps
    t = (np.arange(N) + 0.5) * dt
    return Workload("deform3d", m, a0, Uc, F0, np.full(N, dt), np.cos(np.pi * t / T),
                    meta={"n": n, "T": T, "co": 0.5, "centre": list(centre), "radius": radius})


def slotted_sphere_inside(x, centre=(0.5, 0.75, 0.5), radius=0.15, slot_half=0.025,
                          slot_top=0.85):
    """Ball minus the slot {|x - cx| <= w/2, y <= slot_top} (all z)."""
    c = np.asarray(centre)
    ball = ((x - c) ** 2).sum(-1) <= radius * radius
    slot = (np.abs(x[..., 0] - c[0]) <= slot_half) & (x[..., 1] <= slot_top)
    return ball & ~slot


def generated_volumes(mesh) -> np.ndarray:
    """Cell volumes from the generator's description (boxes, tet vertices)."""
    if mesh.kind == "hex":
        return np.prod(mesh.cell_hi - mesh.cell_lo, axis=1)
    p = mesh.points[mesh.cell_verts]
    return np.abs(np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]),
                            p[:, 3] - p[:, 0])) / 6.0


def max_cell_courant_rate(mesh, F0) -> float:
    """max over cells of (1/2) sum_f |F_f| / V_c: the cell Courant number of a
    unit time step (the outflow volume of a divergence-free cell over its
    volume)."""
    S = np.zeros(mesh.n_cells)
    a = np.abs(F0)
    np.add.at(S, mesh.owner, a)
    np.add.at(S, mesh.neighbour, a[:mesh.n_internal])
    return float((0.5 * S / generated_volumes(mesh)).max())


def rotate_tets(n: int = 80, steps: int | None = None, seed: int = 1305,
                sample: int = 12, centre=(0.5, 0.75, 0.5), radius: float = 0.15,
                co: float = 0.5) -> Workload:
    """Slotted sphere rotating about z through (0.5, 0.5) on jittered Kuhn tets.

    omega = 2 pi, one revolution per unit time.  The step is the largest
    1/N with every cell's Courant number (1/2) sum_f |F_f| dt / V_c at most
    `co`: the jittered tets hold slivers down to about h^3 / 70, so this is
    far below the step a velocity-over-spacing Courant number would give
    (about 1/(300 n) at n = 80, against 1/(9 n)).  The default step count is
    one revolution.
    """
    m = kuhn_tet_mesh(n, 0.2, seed)
    c = np.asarray(centre, dtype=np.float64)
    a0 = fields.tet_fraction_sampled(
        m, lambda x: slotted_sphere_inside(x, c, radius, slot_top=c[1] + 0.1), sample)
    omega = 2.0 * np.pi
    origin = np.array([0.5, 0.5, 0.5])
    Uc = fields.rotation_velocity(m.cell_centroids(), omega, origin)
    F0 = fields.flux_rotation(m, omega, origin)
    per_rev = int(np.ceil(max_cell_courant_rate(m, F0) / co))
    N = per_rev if steps is None else steps
    dt = 1.0 / per_rev
    return Workload("rotate_tets", m, a0, Uc, F0, np.full(N, dt), np.ones(N),
                    meta={"n": n, "seed": seed, "omega": omega, "centre": list(centre),
                          "radius": radius, "co": co, "steps_per_rev": per_rev})


def translate_slab(n: int = 16, nz: int = 1, a: float = 0.3, b: float = 0.55,
                   U=(0.25, 0.0, 0.0), steps: int = 8, dt: float | None = None) -> Workload:
    """Axis-aligned slab {a < x < b} moved along +x by a uniform velocity.

    The exact solution after k steps is the cell fraction of
    {a + u t_k < x < b + u t_k}; used as a whole-step closed form.
    """
    m = hex_mesh(n, n, nz, (0.0, 0.0, 0.0), (1.0, 1.0, nz / n))
    lo, hi = m.cell_lo[:, 0], m.cell_hi[:, 0]
    a0 = np.clip((np.minimum(hi, b) - np.maximum(lo, a)) / (hi - lo), 0.0, 1.0)
    U = np.asarray(U, dtype=np.float64)
    Uc = np.broadcast_to(U, (m.n_cells, 3)).copy()
    F0 = fields.flux_constant(m, U)
    if dt is None:
        dt = 0.5 / n / np.linalg.norm(U)
    return Workload("slab", m, a0, Uc, F0, np.full(steps, dt), np.ones(steps),
                    meta={"a": a, "b": b, "U": U.tolist(), "n": n})


def slab_exact(w: Workload, k: int) -> np.ndarray:
    """Exact cell fractions of the translated slab after k steps."""
    t = float(np.sum(w.dt[:k] * w.scale[:k]))
    u = w.meta["U"][0]
    a = w.meta["a"] + u * t
    b = w.meta["b"] + u * t
    lo, hi = w.mesh.cell_lo[:, 0], w.mesh.cell_hi[:, 0]
    return np.clip((np.minimum(hi, b) - np.maximum(lo, a)) / (hi - lo), 0.0, 1.0)


def courant_schedule(Umax: float, h: float, T: float, co: float = 0.5, growth: float = 2.0,
                     steps: int | None = None):
    """Adaptive time steps for a field U0(x) cos(pi t / T) (Section 4.2.2): the
    Courant number of the current step, from the largest velocity of that step
    (at t_n + dt_n / 2), sets the next step to meet `co` again:
    dt_{n+1} = co h / (Umax |cos(pi (t_n + dt_n/2) / T)|).  The step never
    exceeds `growth` times the first one (the field vanishes at t = T/2, where
    the rule alone is unbounded), and the last step ends at T exactly.
    Returns (dt, scale) with scale_n = cos(pi (t_n + dt_n/2) / T)."""
    dt0 = co * h / Umax
    dts, scs = [], []
    t, dt = 0.0, dt0
    while True:
        if steps is None and t + dt >= T * (1.0 - 1e-12):
            dt = T - t
        s = np.cos(np.pi * (t + 0.5 * dt) / T)
        dts.append(dt)
        scs.append(s)
        t += dt
        if (steps is not None and len(dts) == steps) or (steps is None and t >= T * (1.0 - 1e-12)):
            break
        dt = min(co * h / (Umax * max(abs(s), 1e-300)), growth * dt0)
    return np.array(dts), np.array(scs)


def shear3d(n: int = 64, steps: int | None = None, T: float = 3.0, co: float = 0.5,
            centre=(0.5, 0.75, 0.25), radius: float = 0.15, growth: float = 2.0) -> Workload:
    """Sphere in the shear field (eq. 4.5) with the adaptive Courant time step.

    Umax is the largest |U0| at the cell centroids.  The default runs to T."""
    m = hex_mesh(n, n, n)
    a0 = fields.ball_box_fraction(centre, radius, m.cell_lo, m.cell_hi)
    Uc = fields.shear_velocity(m.cell_centroids())
    F0 = fields.flux_shear(m)
    Umax = float(np.linalg.norm(Uc, axis=1).max())
    dt, sc = courant_schedule(Umax, 1.0 / n, T, co, growth, steps)
    return Workload("shear3d", m, a0, Uc, F0, dt, sc,
                    meta={"n": n, "T": T, "co": co, "centre": list(centre), "radius": radius,
                          "Umax": Umax, "growth": growth})


def deform3d_refined(n: int = 32, steps: int | None = None, T: float = 3.0,
                     centre=(0.35, 0.35, 0.35), radius: float = 0.15) -> Workload:
    """The deformation case on an n^3 hex mesh refined once (2:1, hanging
    points) in the cells the sphere's surface cuts; alpha^0 the exact sphere
    fractions of the refined cells, dt = 1/(8n) (Co 0.5 on the fine cells).
    meta["parent"] maps each cell to its cell of the uniform mesh."""
    from .refine import refine_hex
    m0 = hex_mesh(n, n, n)
    f0 = fields.ball_box_fraction(centre, radius, m0.cell_lo, m0.cell_hi)
    m, parent, children = refine_hex(n, (f0 > 0) & (f0 < 1))
    a0 = fields.ball_box_fraction(centre, radius, m.cell_lo, m.cell_hi)
    Uc = fields.deformation_velocity(m.cell_centroids())
    F0 = fields.flux_deformation(m)
    dt = 1.0 / (8 * n)
    N = int(round(T / dt)) if steps is None else steps
    t = (np.arange(N) + 0.5) * dt
    return Workload("deform3d_refined", m, a0, Uc, F0, np.full(N, dt), np.cos(np.pi * t / T),
                    meta={"n": n, "T": T, "co": 0.5, "centre": list(centre), "radius": radius,
                          "parent": parent, "children": children})


def uniform_alpha(w: Workload, value: float = 0.37) -> Workload:
    """`w` with alpha = value in every cell: every cell is then an interface
    cell whose gradient vanishes (the reconstruction's homogeneous case), so
    every face with flux is clipped and carries value times its swept volume."""
    import dataclasses
    return dataclasses.replace(w, name=w.name + "-uniform", alpha0=np.full(w.mesh.n_cells, value),
                               meta={**w.meta, "uniform": value})


def isolated_cell(n: int = 8, u: float = 0.25, alpha: float = 0.5, steps: int = 1) -> Workload:
    """One cell of value `alpha` at the centre of an empty n^3 box, translated
    along +x at u (Co 0.5): its gradient vanishes by symmetry."""
    m = hex_mesh(n, n, n)
    a0 = np.zeros(m.n_cells)
    c = n // 2
    centre = (c * n + c) * n + c  # cell (c, c, c), x fastest
    a0[centre] = alpha
    U = np.array([u, 0.0, 0.0])
    Uc = np.broadcast_to(U, (m.n_cells, 3)).copy()
    F0 = fields.flux_constant(m, U)
    dt = 0.5 / n / u
    return Workload("isolated_cell", m, a0, Uc, F0, np.full(steps, dt), np.ones(steps),
                    meta={"n": n, "u": u, "alpha": alpha, "cell": centre})


def scaled_translation(n: int = 8, k: float = 20.0, u: float = 0.02, alpha: float = 0.37,
                       steps: int = 1) -> Workload:
    """Uniform translation along +x at u with every face flux k times U.S_f:
    the swept volume is linear in the sweep factor, so the flux correction
    must move the swept points k times the plain sweep (dt = h / 2)."""
    m = hex_mesh(n, n, n)
    U = np.array([u, 0.0, 0.0])
    Uc = np.broadcast_to(U, (m.n_cells, 3)).copy()
    F0 = k * fields.flux_constant(m, U)
    dt = 0.5 / n
    return Workload("scaled_translation", m, np.full(m.n_cells, alpha), Uc, F0,
                    np.full(steps, dt), np.ones(steps), meta={"n": n, "k": k, "u": u})


def courant_dt(mesh, F0, co: float = 0.5, period: float | None = None) -> float:
    """Largest step with every cell's Courant number (1/2) sum_f |F_f| dt / V_c
    at most `co`; with `period`, the largest period / N below it."""
    dt = co / max_cell_courant_rate(mesh, F0)
    if period is not None:
        dt = period / np.ceil(period / dt)
    return float(dt)


def random_unit_vector(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def rotating_sphere(n: int, rng, refine: bool = False, steps: int = 100,
                    r_range=(0.1, 0.2), omega_range=(np.pi, 2 * np.pi)) -> Workload:
    """One instance of the batched workload: a sphere of radius r ~ U(r_range)
    on an n^3 hex mesh (refined once, 2:1, in the cells its surface cuts when
    `refine`), centred uniformly in the ball |c - o| <= 0.5 - r - 2h about
    o = (1/2, 1/2, 1/2), rigidly rotating about o around a uniformly random
    axis at omega ~ U(omega_range); dt from the cell Courant number 0.5 on
    the (finest) cells; exact sphere fractions as alpha^0."""
    from .refine import refine_hex
    h = 1.0 / n
    r = float(rng.uniform(*r_range))
    o = np.array([0.5, 0.5, 0.5])
    rad = max(0.5 - r - 2 * h, 0.0)
    while True:  # uniform in the ball of radius rad
        c = rng.uniform(-rad, rad, size=3) if rad > 0 else np.zeros(3)
        if (c * c).sum() <= rad * rad:
            break
    c = o + c
    axis = random_unit_vector(rng)
    omega = float(rng.uniform(*omega_range))
    m0 = hex_mesh(n, n, n)
    if refine:
        f0 = fields.ball_box_fraction(c, r, m0.cell_lo, m0.cell_hi)
        m, _, _ = refine_hex(n, (f0 > 0) & (f0 < 1))
    else:
        m = m0
    a0 = fields.ball_box_fraction(c, r, m.cell_lo, m.cell_hi)
    Uc = fields.rotation_velocity(m.cell_centroids(), omega, o, axis)
    F0 = fields.flux_rotation(m, omega, o, axis)
    dt = courant_dt(m, F0)
    return Workload(f"sphere{n}{'r' if refine else ''}", m, a0, Uc, F0, np.full(steps, dt),
                    np.ones(steps), meta={"n": n, "refined": refine, "radius": r,
                                          "centre": c.tolist(), "axis": axis.tolist(),
                                          "omega": omega})


def batch_instances(count: int = 256, seed: int = 3417, n_range=(16, 96), steps: int = 100,
                    first: int = 0, stop: int | None = None):
    """The batched workload's instances first .. stop - 1 of `count`: instance
    i has N ~ U{n_range} (one seeded draw per instance) and is refined when i
    is odd (see rotating_sphere).  Every instance draws from its own seeded
    generator, so any subset can be built independently."""
    out = []
    for i in range(first, count if stop is None else stop):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        out.append(rotating_sphere(n, rng, refine=bool(i % 2), steps=steps))
    return out


def sphere_fraction(mesh, centre, radius, sample: int = 6) -> np.ndarray:
    """alpha^0 of a ball on a generated mesh: exact on boxes, sampled on tets."""
    if mesh.kind == "hex":
        return fields.ball_box_fraction(centre, radius, mesh.cell_lo, mesh.cell_hi)
    c = np.asarray(centre, dtype=np.float64)
    return fields.tet_fraction_sampled(
        mesh, lambda x: ((x - c) ** 2).sum(-1) <= radius * radius, sample)


def deformation_template(kind: str, n: int, T: float = 3.0, seed: int = 1305) -> Workload:
    """A mesh of the served workload in the deformation field (eq. 4.6):
    kind "hex" (n^3 cubes) or "tets" (n^3 cubes of six jittered tets); the
    step from the cell Courant number 0.5 (T / N); alpha0 and the schedule
    come with each request (served_request)."""
    m = hex_mesh(n, n, n) if kind == "hex" else kuhn_tet_mesh(n, 0.2, seed)
    Uc = fields.deformation_velocity(m.cell_centroids())
    F0 = fields.flux_deformation(m)
    dt = courant_dt(m, F0, 0.5, T)
    return Workload(f"{kind}{n}", m, np.zeros(m.n_cells), Uc, F0, np.array([dt]), np.ones(1),
                    meta={"kind": kind, "n": n, "T": T})


def served_request(tpl: Workload, rng, steps: int, r_range=(0.1, 0.2)):
    """One request on a template: a sphere r ~ U(r_range) centred in
    U[0.3, 0.7]^3, advected `steps` steps from t = 0 in the deformation
    field (scale cos(pi t / T) at mid-step).  Returns (alpha0, dt, scale)."""
    r = float(rng.uniform(*r_range))
    c = rng.uniform(0.3, 0.7, size=3)
    a0 = sphere_fraction(tpl.mesh, c, r)
    dt = float(tpl.dt[0])
    t = (np.arange(steps) + 0.5) * dt
    return a0, np.full(steps, dt), np.cos(np.pi * t / tpl.meta["T"])


def boundary_points(mesh) -> np.ndarray:
    """Points on the faces of the unit box (bool per point)."""
    p = mesh.points
    return ((p == 0.0) | (p == 1.0)).any(axis=1)


WORKLOADS = {"disc2d": disc2d, "deform3d": deform3d, "rotate_tets": rotate_tets,
             "shear3d": shear3d, "deform3d_refined": deform3d_refined}
