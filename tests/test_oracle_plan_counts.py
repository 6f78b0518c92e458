"""Pins of the oracle's plan (subdomains, oversampled boxes, interfaces,
colours) against closed-form counts of the benchmark workloads.

An oversampled box is the subdomain grown by l cells on every side and cut
at the domain boundary (Section 3), so on an M x M partition of S x S
subdomains there are (M - 2)^2 interior boxes of (S + 2l)^2 cells, 4 (M - 2)
edge boxes of (S + l) x (S + 2l) or the transpose, and 4 corner boxes of
(S + l)^2.  The interface system has one flux and one pressure unknown per
basis function of M_H on each coarse interface (Proposition 1): 2 p per
interface, with p = 1 for piecewise-constant and 2 for piecewise-linear
spaces in 2-D, and 2 M (M - 1) interfaces.  These counts are computed here
from the definitions, not by the oracle's code paths they check.
"""
import collections

import numpy as np
import pytest

from inputs import make_workload
from oracle import mrcm


def _census(part):
    shapes = collections.Counter()
    for i in range(part.nsub):
        lo, hi = part.omega_hat(i)
        shapes[tuple(h - l for l, h in zip(lo, hi))] += 1
    return shapes


def _expected_census(M, S, l):
    full, cut = S + 2 * l, S + l
    out = collections.Counter()
    out[(full, full)] += (M - 2) ** 2
    out[(cut, full)] += 2 * (M - 2)
    out[(full, cut)] += 2 * (M - 2)
    out[(cut, cut)] += 4
    return +out  # drops zero counts (l = 0 makes all shapes equal)


@pytest.mark.parametrize("name,overlap", [("c1", None), ("c2", 0), ("c2", 2), ("c2", 4),
                                          ("c3", None), ("c5", None)])
def test_oversampled_box_census(name, overlap):
    wl = make_workload(name, overlap=overlap)
    part = mrcm.Partition(wl.ncell, wl.sub, wl.overlap)
    M, S = wl.ncell[0] // wl.sub[0], wl.sub[0]
    assert part.nsub == M * M
    got = _census(part)
    exp = _expected_census(M, S, wl.overlap)
    if wl.overlap == 0:
        exp = collections.Counter({(S, S): M * M})
    assert got == exp


def test_c3_census_numbers():
    # 64 x 64 subdomains of 16^2 cells, l = 4: 3844 boxes of 24^2, 248 of
    # 20 x 24 or 24 x 20, 4 of 20^2
    wl = make_workload("c3")
    got = _census(mrcm.Partition(wl.ncell, wl.sub, wl.overlap))
    assert got[(24, 24)] == 3844
    assert got[(20, 24)] + got[(24, 20)] == 248
    assert got[(20, 20)] == 4
    assert sum(got.values()) == 4096


@pytest.mark.parametrize("name,p,expected", [("c1", 1, 48), ("c2", 2, 1920), ("c3", 1, 16128),
                                             ("c5", 1, 960)])
def test_interface_dimension(name, p, expected):
    wl = make_workload(name)
    assert {"const": 1, "linear": 2}[wl.space] == p
    part = mrcm.Partition(wl.ncell, wl.sub, wl.overlap)
    M = wl.ncell[0] // wl.sub[0]
    ifc = part.interfaces()
    assert len(ifc) == 2 * M * (M - 1)
    assert 2 * p * len(ifc) == expected
    # each interface joins two neighbours along one axis, lower index first
    for i, a, j in ifc:
        assert i < j and j == part.neighbor(i, 2 * a + 1)


def test_interface_dimension_of_an_assembled_system():
    # the smallest workload end to end: the assembled interface system has
    # the closed-form size
    s = mrcm.MRCM(make_workload("c1"))
    s.build_basis()
    assert s.offset[-1] == 48


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_parity_colours_separate_neighbours(name):
    # 2^d parity colours: no two subdomains of one colour share a side, and
    # every colour has the same number of subdomains on an even partition
    wl = make_workload(name)
    part = mrcm.Partition(wl.ncell, wl.sub, wl.overlap)
    cols = np.array([part.color(i) for i in range(part.nsub)])
    for i in range(part.nsub):
        for q in part.gamma_sides(i):
            assert cols[part.neighbor(i, q)] != cols[i]
    counts = np.bincount(cols, minlength=4)
    assert (counts == part.nsub // 4).all()
