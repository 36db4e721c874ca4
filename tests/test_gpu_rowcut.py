"""GPU parity of the row cuts.

The contact search orders each neighbour row by the gap g = d - (R_i + R_j)
it finds (touching first, then g < s/8, s/4, s/2 of the skin s, then the
rest), and the force kernel reads a row only as far as a device-side bound on
the displacement since the search allows (Sec. 3.1: a pair whose gap was g
cannot touch before the two spheres have moved g between them).  These tests
make the bound tight and check, step by step with no search in between, that
every contact is found at the step the oracle finds it.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_from_scene

pytestmark = pytest.mark.gpu

D = 3.0e-3           # sphere diameter
SKIN = 0.3 * D       # r_s - d_max at the threshold 1.3
DT = 1.0e-5
SPEED = 0.5          # every sphere moves at this speed until its contact


@pytest.fixture(scope="module")
def Dem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_09576_amd import Dem as D_
    return D_


def head_on_pairs(gaps):
    """Pairs of spheres approaching head on along z at SPEED each, one pair per
    initial gap, the pairs 10 diameters apart along x.  Every sphere moves at
    the same speed, so the displacement bound grows exactly as fast as the
    pairs close: a pair whose gap lies just above a class edge f s can first
    touch at the step the bound reaches f."""
    pos, vel = [], []
    for k, g in enumerate(gaps):
        x = 10 * D * k
        pos += [[x, 0.0, 0.0], [x, 0.0, D + g]]
        vel += [[0.0, 0.0, SPEED], [0.0, 0.0, -SPEED]]
    pos = np.array(pos)
    lo = (-5 * D, -5 * D, -5 * D)
    hi = (10 * D * len(gaps) + 5 * D, 5 * D, 6 * D)
    return dict(name="rowcut_pairs",
                config=W._cfg(DT, lo, hi, threshold=1.3, K=10 ** 6, gravity=(0.0, 0.0, 0.0)),
                materials=[dict(W.BOX_MATERIAL)], walls=[],
                particles=W._particles(pos, np.full(len(pos), D / 2), np.array(vel)))


EPS = 1e-3 * SKIN
GAPS = [0.02 * SKIN,
        SKIN / 8 - EPS, SKIN / 8 + EPS,
        SKIN / 4 - EPS, SKIN / 4 + EPS,
        SKIN / 2 - EPS, SKIN / 2 + EPS,
        0.6 * SKIN, 0.75 * SKIN]


def touching_pairs(g):
    p, _, t = g.get_contacts()
    return {tuple(r) for r, f in zip(p.tolist(), t.tolist()) if f}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_contacts_start_at_the_oracle_step_at_every_class_edge(Dem, precision):
    sc = head_on_pairs(GAPS)
    g = Dem.from_scene(sc, precision=precision)
    o = oracle_from_scene(sc)
    # the FP32 law changes the bounce, not the approach: compare its contact
    # flags while every pair is still approaching or in its first contact
    n_steps = 80 if precision == "fp64" else 70
    first = {}
    for step in range(1, n_steps + 1):
        g.step(1)
        o.step(1)
        gp, _, gt = g.get_contacts()
        op, _, ot = o.contacts()
        assert np.array_equal(gp, op), step          # no search: the same candidates
        assert np.array_equal(gt, ot), (precision, step)
        for pr in touching_pairs(g):
            first.setdefault(pr, step)
        if precision == "fp64":
            Fg, Tg = g.get_forces()
            Fo, To, S = o.forces()
            scale = np.linalg.norm(Fo, axis=1) + S + 1e-300
            assert np.max(np.linalg.norm(Fg - Fo, axis=1) / scale) <= 1e-11, step
    # every pair touched, the pairs in the order of their gaps
    starts = [first[(2 * k, 2 * k + 1)] for k in range(len(GAPS))]
    print(precision, "first touching step per gap:", starts, flush=True)
    assert len(first) == len(GAPS)
    assert starts == sorted(starts)
    # a pair just above a class edge starts one step after the pair just below
    for k in (1, 3, 5):
        assert starts[k + 1] - starts[k] in (0, 1)


def test_sparse_random_bed_contacts_every_step(Dem):
    """Spheres on a lattice with gaps of a sixth of the skin and random
    velocities collide pair by pair; no search for 40 steps, contact sets and
    forces against the oracle after every step."""
    sc = W.dense_snapshot(n=1728, seed=31, overlap=-0.05, vmax=0.3, wmax=20.0, K=10 ** 6)
    g = Dem.from_scene(sc, precision="fp64")
    o = oracle_from_scene(sc)
    new_contacts = 0
    before = touching_pairs(g)
    for step in range(1, 41):
        g.step(1)
        o.step(1)
        gp, _, gt = g.get_contacts()
        op, _, ot = o.contacts()
        assert np.array_equal(gp, op), step
        assert np.array_equal(gt, ot), step
        now = touching_pairs(g)
        new_contacts += len(now - before)
        before = now
        Fg, Tg = g.get_forces()
        Fo, To, S = o.forces()
        scale = np.linalg.norm(Fo, axis=1) + S + 1e-300
        assert np.max(np.linalg.norm(Fg - Fo, axis=1) / scale) <= 1e-9, step
    print("contacts formed during the 40 steps:", new_contacts, flush=True)
    assert new_contacts > 100
