"""Exact rational geometry used to pin the oracle (fractions.Fraction).

An independent, tiny implementation: a tetrahedron clipped by half-spaces is
kept as a list of tetrahedra; each plane splits every tetrahedron into the
kept tetrahedra of its four sign cases (one vertex kept: a corner tet; three
kept: a prism; two kept: a wedge, each cut into three tets).  With dyadic
inputs every intersection point and volume is exact.
"""
from __future__ import annotations

from fractions import Fraction as Q
from itertools import product


def _q(x):
    """Exact rational of a Python/NumPy number (binary floats are exact)."""
    return x if isinstance(x, Q) else Q(float(x))


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _det(a, b, c):
    return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
            + a[2] * (b[0] * c[1] - b[1] * c[0]))


def tet_volume(t):
    a, b, c, d = t
    v = _det(_sub(b, a), _sub(c, a), _sub(d, a)) / 6
    return v if v >= 0 else -v


def _cut(p, dp, q, dq):
    t = dp / (dp - dq)
    return tuple(p[i] + t * (q[i] - p[i]) for i in range(3))


def clip_tets(tets, n, s):
    """Keep {x : n.x <= s} of every tet in the list."""
    out = []
    for t in tets:
        d = [sum(n[i] * v[i] for i in range(3)) - s for v in t]
        ins = [k for k in range(4) if d[k] <= 0]
        outs = [k for k in range(4) if d[k] > 0]
        if len(ins) == 4:
            out.append(t)
        elif len(ins) == 1:
            a = ins[0]
            out.append((t[a],) + tuple(_cut(t[a], d[a], t[o], d[o]) for o in outs))
        elif len(ins) == 3:
            o = outs[0]
            a, b, c = ins
            ad = _cut(t[a], d[a], t[o], d[o])
            bd = _cut(t[b], d[b], t[o], d[o])
            cd = _cut(t[c], d[c], t[o], d[o])
            out += [(t[a], t[b], t[c], ad), (t[b], t[c], ad, bd), (t[c], ad, bd, cd)]
        elif len(ins) == 2:
            a, b = ins
            c, e = outs
            ac = _cut(t[a], d[a], t[c], d[c])
            ae = _cut(t[a], d[a], t[e], d[e])
            bc = _cut(t[b], d[b], t[c], d[c])
            be = _cut(t[b], d[b], t[e], d[e])
            out += [(t[a], ac, ae, t[b]), (ac, ae, t[b], bc), (ae, t[b], bc, be)]
    return out


def tet_halfspaces_volume(tet, planes):
    tets = [tuple(tuple(_q(x) for x in v) for v in tet)]
    for pl in planes:
        n = tuple(_q(x) for x in pl[:3])
        tets = clip_tets(tets, n, _q(pl[3]))
    return sum((tet_volume(t) for t in tets), Q(0))


def box_planes(lo, hi):
    return [(-1, 0, 0, -lo[0]), (1, 0, 0, hi[0]), (0, -1, 0, -lo[1]), (0, 1, 0, hi[1]),
            (0, 0, -1, -lo[2]), (0, 0, 1, hi[2])]


def truncated_box_volume(m, s, lo=(0, 0, 0), hi=(1, 1, 1)):
    """Exact |box ∩ {m.x <= s}| by inclusion-exclusion over the box corners
    (every m_i != 0): sum_v (-1)^{#upper} max(0, s - m.v)^3 / (6 m1 m2 m3),
    after reflecting negative components."""
    m = [_q(x) for x in m]
    s = _q(s)
    lo = [_q(x) for x in lo]
    hi = [_q(x) for x in hi]
    # reflect so every component is positive
    for i in range(3):
        if m[i] < 0:
            m[i] = -m[i]
            lo[i], hi[i] = -hi[i], -lo[i]
    tot = Q(0)
    for sel in product((0, 1), repeat=3):
        v = [hi[i] if sel[i] else lo[i] for i in range(3)]
        r = s - sum(m[i] * v[i] for i in range(3))
        if r > 0:
            tot += (-1) ** sum(sel) * r ** 3
    return tot / (6 * m[0] * m[1] * m[2])
