"""Parity at full size: the 1,000,000-atom box (100^3 jittered lattice,
C = 128, l_max = 2, K = 2).  The oracle cannot evaluate the whole box in
seconds, so it evaluates non-periodic clusters cut around sampled atoms:
with radius 2 K r_c and the energy summed over atoms within K r_c of the
center, the center's force and the energies of all atoms within K r_c are
the exact full-system values (each hop of the message passing is shorter
than r_c).  Properties that hold at any size are checked on all atoms.
Tolerances are those of test_gpu_parity."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
K = 2
CENTERS = (123456, 777777)


@pytest.fixture(scope="module")
def bulk():
    import torch
    import paper_2509_21694_amd as M
    s = W.bulk1m_system()
    blob = W.make_weights(W.HP_BULK, W.WEIGHT_SEEDS["bulk1m"])
    model = M.Model(W.HP_BULK, blob)
    pos = torch.tensor(s.positions, dtype=torch.float64, device="cuda")
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    out = {}
    for prec in ("bf16", "fp32"):
        o = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision=prec, atom_energy=True)
        out[prec] = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in o.items()}
        print(f"bulk1m {prec}: edges={o['n_edges']} E={out[prec]['energy'][0]:.6f}")
    again = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision="bf16")
    out["repeat_equal"] = bool(torch.equal(again["forces"].cpu(), torch.tensor(out["bf16"]["forces"])))
    return s, blob, out


@pytest.fixture(scope="module")
def refs(bulk):
    s, blob, _ = bulk
    rc = W.HP_BULK.r_cut
    res = []
    for a in CENTERS:
        lp, ls, n_in, gi, c = oracle.local_cluster(s.positions, s.species, s.cell, a, 2 * K * rc, K * rc)
        r = oracle.evaluate(lp, ls, np.eye(3), [False] * 3, blob, W.HP_BULK, K=K, n_owned=n_in)
        res.append((a, r.forces[c], gi[:n_in], r.atom_energy[:n_in]))
    return res


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bulk_sampled_parity(bulk, refs, prec):
    s, _, out = bulk
    F = out[prec]["forces"]
    ae = out[prec]["atom_energy"]
    for a, fref, gi, eref in refs:
        dF = np.abs(F[a] - fref)
        dE = np.abs(ae[gi] - eref)
        print(f"[{prec}] atom {a}: |F|={np.linalg.norm(fref):.3e} max|dF|={dF.max():.3e} "
              f"max|dE_i| over {gi.size} atoms={dE.max():.3e}")
        if prec == "fp32":
            assert dF.max() <= 1e-4 and dF.max() <= 1e-5 * max(np.abs(fref).max(), 1e-3)
            assert dE.max() <= 1e-6
        else:
            assert dF.max() <= 5e-3 and dF.max() <= 5e-2 * max(np.abs(fref).max(), 1e-3)
            assert dE.max() <= 1e-3


def test_bulk_invariants(bulk):
    s, _, out = bulk
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
