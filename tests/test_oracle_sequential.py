"""The paper's collision order taken literally (oracle.step_sequential), CPU only.

Sec. "Collision Operator" and Sec. "Particle-Particle Collisions" visit elements
along a space-filling curve and accept the first valid collision a particle
finds among its candidate elements; both particles then leave the eligible set.
This sequential rule is pinned here (a closed-form case where it differs from the
earliest-partner rule, isolated pairs where the two rules coincide bitwise, an
independent pure-Python statement of the same traversal with a bisection root
finder, and the post-conditions of a maximal matching), and compared
statistically with the order-free mutual-earliest rule that the GPU computes."""
import numpy as np
import pytest

import oracle
import workloads
from tests import indep_bruteforce as bf


def _box(pos, vel, r=0.5, L=20.0, dt=3.0, e=1.0):
    pos, vel = np.asarray(pos, float), np.asarray(vel, float)
    n = len(pos)
    return workloads.Box(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), vel[:, 0].copy(),
                         vel[:, 1].copy(), vel[:, 2].copy(), np.full(n, r), np.ones(n),
                         (L, L, L), dt, e)


def test_first_found_is_not_the_earliest():
    # A at rest; B (index 1) reaches it at t = 2, C (index 2) at t = 0.5.  All three
    # share a cell, so A scans B first and takes it; the earliest-partner rule pairs A
    # with C.  With C's index below B's, both rules pair A with C.
    A, B, C = ([5, 5, 5], [0, 0, 0]), ([8, 5, 5], [-1, 0, 0]), ([3.5, 5, 5], [1, 0, 0])
    box = _box([A[0], B[0], C[0]], [A[1], B[1], C[1]])
    seq, mut = oracle.step_sequential(box), oracle.step(box)
    assert seq.n_pairs == 1 and seq.partner[0] == 1 and seq.tcoll[0] == 2.0
    assert seq.partner[2] == -1
    assert mut.n_pairs == 1 and mut.partner[0] == 2 and mut.tcoll[0] == 0.5
    box2 = _box([A[0], C[0], B[0]], [A[1], C[1], B[1]])
    seq2, mut2 = oracle.step_sequential(box2), oracle.step(box2)
    assert seq2.partner[0] == 1 == mut2.partner[0] and seq2.tcoll[0] == 0.5


def test_isolated_pairs_equal_the_mutual_rule_bitwise():
    # pairs on a coarse lattice, each closing head-on with a random offset; no sphere
    # can reach a sphere of another pair within the step
    rng = np.random.default_rng(8)
    pos, vel = [], []
    for i in range(6):
        for j in range(6):
            for k in range(6):
                c = np.array([i, j, k]) * 10.0 + 5.0
                dirn = rng.normal(size=3)
                dirn /= np.linalg.norm(dirn)
                off = rng.normal(size=3) * 0.2
                pos += [c - 1.5 * dirn, c + 1.5 * dirn + off]
                vel += [dirn * 0.5, -dirn * 0.5]
    box = _box(pos, vel, L=60.0, dt=2.5, e=0.8)
    seq, mut = oracle.step_sequential(box), oracle.step(box)
    assert mut.n_pairs > 150 and mut.n_sweeps == 2
    assert np.array_equal(seq.partner, mut.partner)
    assert np.array_equal(seq.tcoll, mut.tcoll, equal_nan=True)
    for f in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(getattr(seq, f).view(np.uint64), getattr(mut, f).view(np.uint64))


def _morton(c):
    k = 0
    for b in range(21):
        for a in range(3):
            k |= ((c[a] >> b) & 1) << (3 * b + a)
    return k


def _literal_bruteforce(box):
    """The literal traversal in plain Python with the bisection contact time."""
    n, L = box.n, box.L
    p = [box.x, box.y, box.z]
    vmax = max(np.sqrt(box.vx ** 2 + box.vy ** 2 + box.vz ** 2))
    reach = 2 * max(box.r) + 2 * vmax * box.dt
    nc = [min(max(int(np.floor(L[a] / (reach * (1 + 1e-9)))), 1), 2048) for a in range(3)]
    h = [L[a] / nc[a] for a in range(3)]
    cell_of = [tuple(min(max(int(np.floor(p[a][i] / h[a])), 0), nc[a] - 1) for a in range(3))
               for i in range(n)]
    members = {}
    for i in range(n):
        members.setdefault(cell_of[i], []).append(i)
    cells = sorted(((cx, cy, cz) for cz in range(nc[2]) for cy in range(nc[1])
                    for cx in range(nc[0])), key=_morton)
    hit, pairs = [False] * n, {}
    for c in cells:
        offs = [sorted({(c[a] + o) % nc[a] for o in (-1, 0, 1)}) for a in range(3)]
        cand = sorted(((qx, qy, qz) for qz in offs[2] for qy in offs[1] for qx in offs[0]),
                      key=_morton)
        for i in members.get(c, []):
            if hit[i]:
                continue
            xi, vi = (box.x[i], box.y[i], box.z[i]), (box.vx[i], box.vy[i], box.vz[i])
            for q in cand:
                for j in members.get(q, []):
                    if j == i or hit[j]:
                        continue
                    t = bf.contact_time(xi, vi, box.r[i], (box.x[j], box.y[j], box.z[j]),
                                        (box.vx[j], box.vy[j], box.vz[j]), box.r[j], L, box.dt)
                    if t is None:
                        continue
                    hit[i] = hit[j] = True
                    pairs[(min(i, j), max(i, j))] = t
                    break
                if hit[i]:
                    break
    return pairs


@pytest.mark.parametrize("seed,n,L", [(1, 250, None), (2, 400, None), (3, 600, 40.0),
                                       (4, 900, 48.0)])
def test_matches_independent_literal_traversal(seed, n, L):
    if L is None:
        box = workloads.make_box(n, seed=seed, phi=0.3, radius=0.5, e=0.85, dt=0.25)
    else:  # boxes with three or more cells per axis
        box = workloads.make_box(n, seed=seed, phi=0.2, radius=0.5, e=0.85, dt=0.1)
    res = oracle.step_sequential(box)
    ref = _literal_bruteforce(box)
    got = {(i, int(res.partner[i])): res.tcoll[i] for i in range(box.n) if res.partner[i] > i}
    assert set(got) == set(ref) and len(ref) > 20
    for key in ref:
        assert got[key] == pytest.approx(ref[key], rel=1e-9)


def test_maximal_matching_post_conditions():
    box = workloads.config(2, n=100_000)
    res = oracle.step_sequential(box)
    col = np.nonzero(res.partner >= 0)[0]
    assert res.n_pairs * 2 == len(col) and res.n_pairs > 10_000
    assert np.array_equal(res.partner[res.partner[col]], col)
    for i in col[:2000]:
        j = int(res.partner[i])
        t = oracle.pair_time((box.x[i], box.y[i], box.z[i]), (box.vx[i], box.vy[i], box.vz[i]),
                             box.r[i], (box.x[j], box.y[j], box.z[j]),
                             (box.vx[j], box.vy[j], box.vz[j]), box.r[j], box.L, box.dt)
        assert t is not None and t == res.tcoll[i]
    # no two spheres left free can still collide within the step
    free = (res.partner < 0).astype(np.uint8)
    pj, _, _ = oracle.earliest(box, active=free)
    assert np.all(pj[free.astype(bool)] < 0)


def test_departure_from_the_mutual_earliest_rule():
    """The two rules on the 1M recipe at 100k spheres: the literal one finds a few per
    cent more pairs and dissipates a few per cent more energy per step, and gives a
    different partner to a fifth or more of the colliding spheres; over 30 steps of
    homogeneous cooling the kinetic energies stay within one per cent."""
    box = workloads.config(2, n=100_000)
    seq, mut = oracle.step_sequential(box), oracle.step(box)
    ke = lambda vx, vy, vz: 0.5 * np.sum(box.m * (vx * vx + vy * vy + vz * vz))
    k0 = ke(box.vx, box.vy, box.vz)
    d_seq, d_mut = k0 - ke(seq.vx, seq.vy, seq.vz), k0 - ke(mut.vx, mut.vy, mut.vz)
    assert 0.0 < (seq.n_pairs - mut.n_pairs) / mut.n_pairs < 0.05
    assert 0.0 < (d_seq - d_mut) / d_mut < 0.05
    same = np.sum((seq.partner == mut.partner) & (mut.partner >= 0)) / np.sum(mut.partner >= 0)
    assert 0.5 < same < 0.95
    small = workloads.config(2, n=20_000)
    curves = []
    for rule in (oracle.step, oracle.step_sequential):
        b = small.copy()
        k = [0.5 * np.sum(b.m * (b.vx ** 2 + b.vy ** 2 + b.vz ** 2))]
        for _ in range(30):
            r = rule(b)
            b.x, b.y, b.z, b.vx, b.vy, b.vz = r.x, r.y, r.z, r.vx, r.vy, r.vz
            k.append(0.5 * np.sum(b.m * (b.vx ** 2 + b.vy ** 2 + b.vz ** 2)))
        curves.append(np.array(k) / k[0])
    assert curves[0][-1] < 0.6
    assert np.max(np.abs(curves[1] - curves[0])) < 0.01
