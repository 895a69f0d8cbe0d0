"""Zephyr dimensions the paper states (tests/golden/zephyr_dimensions.json)
against the cell map and projectors used by both the oracle and the HIP path."""
import json
import os

import numpy as np

from tnb_inputs import make_instance
from oracle.potts import Potts, popcount
from oracle.bmps import Network

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "zephyr_dimensions.json")


def _interior_cell(net):
    # a full 16-spin cell whose 8 king neighbours are full cells too (the
    # paper's figures are for a full graph; boundary crosses hold 12 spins)
    for r in range(1, net.R - 1):
        for c in range(1, net.C - 1):
            n = net.cell(r, c)
            nb = [net.cell(r + dr, c + dc) for dr in (-1, 0, 1) for dc in (-1, 0, 1) if (dr, dc) != (0, 0)]
            if net.P.k[n] == 16 and all(net.P.k[m] == 16 for m in nb):
                return r, c
    raise AssertionError("no interior cell")


def test_zephyr_interior_dimensions_match_the_paper():
    g = json.load(open(GOLDEN))
    inst = make_instance("zephyr", 7, jdist="uniform", m=4, t=4)
    net = Network(inst, 1.0)
    r, c = _interior_cell(net)
    n = net.cell(r, c)
    # cluster states
    assert 1 << int(net.P.k[n]) == g["cluster_states"]
    # every projection onto a king neighbour, both ways
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if (dr, dc) == (0, 0):
                continue
            m = net.cell(r + dr, c + dc)
            assert 1 << popcount(net.B(n, m)) == g["projected_dims"][0]
            assert 1 << popcount(net.B(m, n)) == g["projected_dims"][0]
    # site tensor of (r, c): left and right MPO legs, vertical legs to the rows above and below
    site = sorted([1 << popcount(net.PL(r, c)), 1 << popcount(net.PR(r, c)),
                   1 << popcount(net.B(n, net.cell(r - 1, c))), 1 << popcount(net.B(n, net.cell(r + 1, c)))])
    assert site == sorted(g["site_bond_dims"])
    # mediating tensor between (r, c) and (r, c+1): its MPO legs and its two
    # boundary legs (each a pair of diagonal projections)
    dims, split = net.phys_dims(r + 1)
    med = sorted([1 << popcount(net.PR(r, c)), 1 << popcount(net.PL(r, c + 1)),
                  dims[2 * c + 1], net.phys_dims(r)[0][2 * c + 1]])
    assert med == sorted(g["mediating_bond_dims"])


def test_zephyr_typical_degree_matches_the_paper():
    g = json.load(open(GOLDEN))
    inst = make_instance("zephyr", 7, jdist="uniform", m=4, t=4)
    deg = np.bincount(inst.edges.ravel(), minlength=inst.n_spins)
    vals, counts = np.unique(deg, return_counts=True)
    assert vals[np.argmax(counts)] == g["typical_degree"]
