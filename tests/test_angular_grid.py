"""Pins of the oracle's geodesic angular grid (paper Sec. 2.6).

Each check is fixed by the paper or by geometry, not by the oracle itself:
cell counts 10 N^2 + 2 with 12 pentagons (the paper's counts 12, 42, 92,
162, 2252, 4842), the level-1 grid being the regular dodecahedron (closed
form), every polygon's area re-derived by Girard's theorem (a route
independent of the oracle's triangle fan), and the icosahedral symmetry that
makes the first moment vanish and the second isotropic.
"""
import math

import numpy as np
import pytest

from oracle import angular_grid as AG


@pytest.mark.parametrize("nlev", [1, 2, 3, 4, 5, 6, 15, 22])
def test_counts_and_total_solid_angle(nlev):
    g = AG.build(nlev)
    assert g.nang == 10 * nlev * nlev + 2
    k = np.array([len(p) for p in g.polys])
    assert (k == 5).sum() == 12
    assert (k == 6).sum() == g.nang - 12
    assert len(g.lo) == 30 * nlev * nlev
    # every cell has as many edges as polygon corners
    deg = np.bincount(np.concatenate([g.lo, g.hi]), minlength=g.nang)
    assert np.array_equal(deg, k)
    assert abs(g.domega.sum() - 4.0 * math.pi) <= 1e-13


def test_paper_counts():
    # the grid sizes the paper quotes (tests/golden/paper_values.json)
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "paper_values.json")))["geodesic_counts"]
    for nlev, n in zip(gold["levels"], gold["nang"]):
        assert 10 * nlev * nlev + 2 == n
        if nlev <= 4:
            assert AG.build(nlev).nang == n


def test_level1_is_dodecahedron():
    g = AG.build(1)
    assert np.allclose(g.domega, math.pi / 3.0, rtol=0, atol=1e-14)
    # adjacent dodecahedron vertices subtend arccos(sqrt5/3)
    assert np.allclose(g.length, math.acos(math.sqrt(5.0) / 3.0), rtol=0, atol=1e-14)
    # cell centres are the icosahedron's vertices: nearest pairs at cos = 1/sqrt5
    assert abs((g.nhat @ g.nhat.T)[np.triu_indices(12, 1)].max() - 1.0 / math.sqrt(5.0)) < 1e-14


def _girard_area(P):
    k = len(P)
    s = 0.0
    for i in range(k):
        a, b, c = P[i - 1], P[i], P[(i + 1) % k]
        # interior angle at b between great-circle arcs b->a and b->c
        ta = a - b * np.dot(a, b)
        tc = c - b * np.dot(c, b)
        s += math.atan2(np.linalg.norm(np.cross(ta, tc)), np.dot(ta, tc))
    return s - (k - 2) * math.pi


@pytest.mark.parametrize("nlev", [2, 4, 6])
def test_girard_areas(nlev):
    g = AG.build(nlev)
    gir = np.array([_girard_area(P) for P in g.polys])
    assert np.max(np.abs(gir - g.domega)) <= 1e-12


@pytest.mark.parametrize("nlev", [1, 2, 3, 4, 6])
def test_icosahedral_moments(nlev):
    g = AG.build(nlev)
    m1 = (g.domega[:, None] * g.nhat).sum(0)
    m2 = np.einsum("n,ni,nj->ij", g.domega, g.nhat, g.nhat)
    assert np.abs(m1).max() <= 1e-14
    assert np.abs(m2 - 4.0 * math.pi / 3.0 * np.eye(3)).max() <= 1e-13


@pytest.mark.parametrize("nlev", [2, 3])
def test_edges(nlev):
    g = AG.build(nlev)
    assert np.allclose(np.linalg.norm(g.nu, axis=1), 1.0)
    assert np.allclose(np.linalg.norm(g.mid, axis=1), 1.0)
    # normal tangent at the midpoint, pointing from lo towards hi
    assert np.abs(np.einsum("ei,ei->e", g.nu, g.mid)).max() <= 1e-14
    assert (np.einsum("ei,ei->e", g.nu, g.nhat[g.hi] - g.nhat[g.lo]) > 0).all()
    assert (g.lo < g.hi).all()
    # edge lengths add up to each polygon's perimeter
    per = np.zeros(g.nang)
    np.add.at(per, g.lo, g.length)
    np.add.at(per, g.hi, g.length)
    perim = np.array([sum(math.atan2(np.linalg.norm(np.cross(P[i], P[(i + 1) % len(P)])),
                                     np.dot(P[i], P[(i + 1) % len(P)]))
                          for i in range(len(P))) for P in g.polys])
    assert np.allclose(per, perim, rtol=0, atol=1e-13)


def test_canonical_order():
    g = AG.build(3)
    assert np.allclose(g.nhat[0], [0, 0, 1])
    assert np.allclose(g.nhat[-1], [0, 0, -1])
    assert (np.diff(g.nhat[:, 2]) <= 1e-12).all()
