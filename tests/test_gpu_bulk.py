"""Parity at the 1M-atom workload's potential (C = 128, l_max = 2, K = 2),
where the specialised kernels run at C = 128 in their multi-row,
XCD-sliced walk.

* A 32,768-atom periodic box (32^3 jittered lattice, same density, species
  mix and potential): every atom's energy and force, the total energy and the
  stress against the oracle's values (tests/golden/bulk32k_K2.npz).
* The 1,000,000-atom box itself: the oracle cannot evaluate it whole, so it
  evaluated non-periodic clusters of radius 24 A cut around eight atoms spread
  over the box (tests/golden/bulk1m_clusters.npz): with the energy summed over
  the atoms within radius - K r_c, those atoms' energies are the full-system
  values, and so are the forces of the atoms within radius - 2 K r_c (each
  message hop is shorter than r_c).  Properties that hold at any size are
  checked on all atoms.
Tolerances are those of test_gpu_parity."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
K = 2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def model():
    import paper_2509_21694_amd as M
    return M.Model(W.HP_BULK, W.make_weights(W.HP_BULK, W.WEIGHT_SEEDS["bulk1m"]))


@pytest.fixture(scope="module")
def bulk(model):
    import torch
    s = W.bulk1m_system()
    pos = torch.tensor(s.positions, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    out = {}
    for prec in ("bf16", "fp32"):
        o = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision=prec, atom_energy=True)
        out[prec] = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in o.items()}
        print(f"bulk1m {prec}: edges={o['n_edges']} E={out[prec]['energy'][0]:.6f}", flush=True)
    again = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision="bf16")
    out["repeat_equal"] = bool(torch.equal(again["forces"].cpu(), torch.tensor(out["bf16"]["forces"])))
    return s, out


def check(prec, dF, fref, dE_atoms, label):
    frms = np.sqrt(np.mean(fref ** 2))
    rms = np.sqrt(np.mean(dF ** 2))
    print(f"[{label}] {prec}: max|dF|={np.abs(dF).max():.3e} rms dF={rms:.3e} (|F|max={np.abs(fref).max():.3e} "
          f"rms={frms:.3e}, {fref.shape[0]} atoms) max|dE_i|={np.abs(dE_atoms).max():.3e} "
          f"({dE_atoms.size} atoms)")
    if prec == "fp32":
        assert np.abs(dF).max() <= 1e-4 and np.abs(dF).max() <= 1e-5 * np.abs(fref).max()
        assert np.abs(dE_atoms).max() <= 1e-6
    else:
        assert rms <= 5e-3 and rms <= 2e-2 * frms
        assert np.abs(dE_atoms).max() <= 1e-3


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bulk32k_every_atom(model, prec):
    import torch
    g = np.load(os.path.join(GOLDEN, "bulk32k_K2.npz"))
    s = W.bulk_system(32, 311, 312)
    pos = torch.tensor(s.positions, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    o = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision=prec, atom_energy=True)
    assert o["n_edges"] == int(g["n_edges"])
    F = o["forces"].cpu().numpy()
    ae = o["atom_energy"].cpu().numpy()
    check(prec, F - g["forces"], g["forces"], ae - g["atom_energy"], "bulk32k")
    dE = abs(float(o["energy"].cpu()[0]) - float(g["energy"])) / s.n_atoms
    vol = float(np.prod(np.diag(s.cell)))
    dW = np.abs(o["virial"].cpu().numpy() - g["virial"]).max() / vol
    print(f"[bulk32k] {prec}: |dE|/N={dE:.3e} max|dW|/V={dW:.3e} eV/A^3 "
          f"(|W|max/V={np.abs(g['virial']).max() / vol:.3e})")
    assert dE <= (1e-6 if prec == "fp32" else 1e-3)
    assert dW <= (1e-8 if prec == "fp32" else 1e-5)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bulk1m_cluster_parity(bulk, prec):
    s, out = bulk
    g = np.load(os.path.join(GOLDEN, "bulk1m_clusters.npz"))
    F = out[prec]["forces"]
    ae = out[prec]["atom_energy"]
    fi, ei = g["force_index"], g["energy_index"]
    assert fi.size >= 32 and np.unique(g["force_center"]).size == 8
    check(prec, F[fi] - g["forces"], g["forces"], ae[ei] - g["atom_energy"], "bulk1m clusters")


def test_bulk_invariants(bulk):
    s, out = bulk
    for prec in ("fp32", "bf16"):
        o = out[prec]
        F = o["forces"]
        assert np.all(np.isfinite(F))
        # translation invariance: the forces sum to zero
        net = np.abs(F.sum(axis=0)).max()
        print(f"[{prec}] |sum F|={net:.3e} rms F={np.sqrt(np.mean(F ** 2)):.3e}")
        assert net <= (1e-6 if prec == "fp32" else 1e-3)
        # the energy is the sum of the per-atom energies
        assert abs(o["energy"][0] - o["atom_energy"].sum()) <= 1e-6 * max(1.0, abs(o["energy"][0]))
        Wv = o["virial"].reshape(3, 3)
        assert np.abs(Wv - Wv.T).max() <= (1e-6 if prec == "fp32" else 1e-2) * max(1.0, np.abs(Wv).max())
    assert out["fp32"]["n_edges"] == out["bf16"]["n_edges"]
    assert out["repeat_equal"]
