"""Host-side checks of the bisection refinement (Sections 4.2, 4.3: meshes
refined adaptively), through the C interface, no GPU.

A refined mesh must stay a conforming tetrahedrization of the unit cube:
positive volumes summing to 1, every face shared by at most two
tetrahedra, a face of one tetrahedron only lying in the cube's boundary,
Dirichlet flags exactly on the boundary, and the midpoint of every bisected
edge a vertex.  Repeated refinement keeps finitely many shapes (Kuhn
bisection): the ratio of longest edge to inradius stays bounded.
"""
import os

import numpy as np
import pytest

import ocp_inputs as I


def _capi():
    from paper_2102_03515_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libocpamg.so not built")
    return capi


def _check_conforming(xyz, tets, dirichlet):
    p = xyz[tets]
    vol = np.abs(np.linalg.det(p[:, 1:] - p[:, :1])) / 6.0
    assert vol.min() > 0.0
    assert abs(vol.sum() - 1.0) < 1e-12
    faces = np.sort(np.concatenate([np.delete(tets, a, axis=1) for a in range(4)]), axis=1)
    u, c = np.unique(faces, axis=0, return_counts=True)
    assert c.max() <= 2
    bf = xyz[u[c == 1]]                       # [nb,3,3]
    on_plane = np.zeros(len(bf), dtype=bool)
    for ax in range(3):
        for val in (0.0, 1.0):
            on_plane |= np.all(np.abs(bf[:, :, ax] - val) < 1e-14, axis=1)
    assert on_plane.all(), "a face of one tetrahedron inside the cube (hanging node)"
    on_bd = np.any((np.abs(xyz) < 1e-14) | (np.abs(xyz - 1.0) < 1e-14), axis=1)
    np.testing.assert_array_equal(dirichlet.astype(bool), on_bd)
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    L = np.max([np.linalg.norm(p[:, a] - p[:, b], axis=1) for a, b in edges], axis=0)
    area = sum(0.5 * np.linalg.norm(np.cross(p[:, b] - p[:, a], p[:, c] - p[:, a]), axis=1)
               for a, b, c in [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)])
    inradius = 3.0 * vol / area
    return float((L / inradius).max())


def test_local_refinement_stays_conforming():
    capi = _capi()
    m = I.kuhn_mesh(4)
    r = capi.Refiner(m.xyz, m.tets)
    xyz, tets, d = r.get()
    np.testing.assert_array_equal(tets, m.tets)
    np.testing.assert_array_equal(d, m.dirichlet)
    q0 = _check_conforming(xyz, tets, d)
    ratios = []
    for it in range(14):
        c = xyz[tets].mean(axis=1)
        # an indicator that peaks at an interior point off the lattice
        eta2 = np.exp(-60 * np.sum((c - np.array([0.31, 0.47, 0.62])) ** 2, axis=1))
        marked = r.refine(eta2, 0.5)
        assert marked >= 1
        xyz, tets, d = r.get()
        ratios.append(_check_conforming(xyz, tets, d))
    assert len(tets) > 10 * m.n_tets
    # shape classes of Kuhn bisection: the quality measure stays bounded
    assert max(ratios) < 4 * q0
    # every vertex added is the midpoint of an edge of a coarser tetrahedron:
    # new vertices have dyadic coordinates
    assert np.all(np.abs(xyz * 2 ** 12 - np.round(xyz * 2 ** 12)) < 1e-9)


def test_uniform_marking_bisects_everything_and_errors():
    capi = _capi()
    m = I.kuhn_mesh(2)
    r = capi.Refiner(m.xyz, m.tets)
    for k in range(3):     # theta = 1 marks every tetrahedron
        nt0 = r.get()[1].shape[0]
        r.refine(np.ones(nt0), 1.0)
        xyz, tets, d = r.get()
        assert tets.shape[0] == 2 * nt0
        _check_conforming(xyz, tets, d)
    # three bisections of every Kuhn tetrahedron: 8 children of half the diameter
    assert tets.shape[0] == 8 * m.n_tets
    with pytest.raises(capi.OcpError):
        r.refine(np.ones(tets.shape[0]), 0.0)
    with pytest.raises(capi.OcpError):
        r.refine(np.full(tets.shape[0], np.nan), 0.5)
    bad = m.tets.copy()
    bad[0, 0] = 10 ** 6
    with pytest.raises(capi.OcpError):
        capi.Refiner(m.xyz, bad)


@pytest.mark.parametrize("N,jit,steps", [(3, 0.0, 10), (4, 0.15, 6)])
def test_refiner_matches_oracle_bisection(N, jit, steps):
    """The library's refinement equals the oracle's (oracle/refine.py, the
    definition written out in Python) bit for bit: same vertices in the same
    order, same tetrahedra and tags' consequences, same Dirichlet flags, for
    a seeded indicator with distinct values (so the marking is unique)."""
    capi = _capi()
    from oracle.refine import Refiner as OracleRefiner
    m = I.kuhn_mesh(N, jitter=jit, seed=9)
    r = capi.Refiner(m.xyz, m.tets)
    o = OracleRefiner(m.xyz, m.tets)
    rng = np.random.default_rng(10)
    for k in range(steps):
        xyz, tets, d = r.get()
        oxyz, otets, od = o.mesh()
        np.testing.assert_array_equal(tets, otets)
        np.testing.assert_array_equal(xyz, oxyz)
        np.testing.assert_array_equal(d, od)
        c = xyz[tets].mean(axis=1)
        eta2 = np.exp(-30 * np.sum((c - 0.4) ** 2, axis=1)) * (1.0 + 0.01 * rng.random(len(tets)))
        assert r.refine(eta2, 0.4) == o.refine(eta2, 0.4)


def test_oracle_bisection_is_conforming():
    """The oracle's refinement by itself: conforming, volumes summing to 1,
    Dirichlet flags exactly on the cube's boundary."""
    from oracle.refine import Refiner as OracleRefiner
    m = I.kuhn_mesh(3)
    o = OracleRefiner(m.xyz, m.tets)
    for k in range(8):
        xyz, tets, d = o.mesh()
        _check_conforming(xyz, tets, d)
        c = xyz[tets].mean(axis=1)
        o.refine(np.exp(-40 * np.sum((c - 0.7) ** 2, axis=1)), 0.5)
