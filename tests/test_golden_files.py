"""Integrity of the stored oracle outputs the GPU parity tests compare
against (written by tests/golden/make_golden.py from the oracle alone):
shapes, the energy as the sum of atom energies, zero net force, a symmetric
virial, and for the 1M-atom clusters the sampling the parity test relies on
(eight centers, every force atom within 4 A of its center)."""
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_bulk32k_golden_consistent():
    g = np.load(os.path.join(GOLDEN, "bulk32k_K2.npz"))
    n = 32 ** 3
    assert g["forces"].shape == (n, 3) and g["atom_energy"].shape == (n,)
    assert abs(float(g["energy"]) - g["atom_energy"].sum()) <= 1e-9 * abs(float(g["energy"]))
    assert np.abs(g["forces"].sum(axis=0)).max() <= 1e-10
    Wv = g["virial"]
    assert np.abs(Wv - Wv.T).max() <= 1e-10 * np.abs(Wv).max()
    # mean degree of the jittered lattice at 5 A: about 38 directed edges per atom
    assert 36 * n <= int(g["n_edges"]) <= 41 * n


def test_bulk1m_cluster_golden_layout():
    g = np.load(os.path.join(GOLDEN, "bulk1m_clusters.npz"))
    centers = g["centers"]
    assert centers.size == 8 and np.unique(g["force_center"]).size == 8
    assert g["forces"].shape == (g["force_index"].size, 3)
    assert g["atom_energy"].shape == g["energy_index"].shape
    # every force atom lies within radius - 2 K r_c = 4 A (minimum image) of its center
    s = W.bulk1m_system()
    L = np.diag(s.cell)
    d = s.positions[g["force_index"]] - s.positions[g["force_center"]]
    d -= np.round(d / L) * L
    assert np.sqrt((d ** 2).sum(axis=1)).max() <= float(g["radius"]) - 2 * 2 * W.HP_BULK.r_cut
    assert g["force_index"].size >= 32
