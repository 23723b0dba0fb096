"""Batched evaluation of 512 independent small periodic cells (8..512 atoms,
sides 6-20 A or thinner cubes below 216 A^3, 3 species, l_max = 2, C = 64,
K = 2) in one pass of every kernel: per-structure energies, forces and
virials against the FP64 oracle on a sample of structures (the smallest,
the largest and a seeded random subset), and properties on all of them.
Tolerances are those of test_gpu_parity."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch_case():
    import torch
    import paper_2509_21694_amd as M
    structs = W.batch_structures()
    hp = W.HP_BATCH
    blob = W.make_weights(hp, W.WEIGHT_SEEDS["batch512"])
    model = M.Model(hp, blob)
    batch = M.Batch(structs, torch.device("cuda", 0))
    out = {}
    for prec in ("fp32", "bf16"):
        o = M.evaluate_batch(model, batch, K=2, precision=prec)
        out[prec] = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in o.items()}
    sizes = np.diff(batch.atom_ptr)
    rng = np.random.default_rng(7)
    pick = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes))] + rng.choice(len(structs), 10, replace=False).tolist()))
    refs = {b: oracle.evaluate(structs[b].positions, structs[b].species, structs[b].cell, structs[b].pbc, blob, hp, K=2)
            for b in pick}
    return structs, batch, out, refs


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_parity(batch_case, prec):
    structs, batch, out, refs = batch_case
    o = out[prec]
    for b, ref in refs.items():
        a0, a1 = batch.atom_ptr[b], batch.atom_ptr[b + 1]
        n = a1 - a0
        F = o["forces"][a0:a1]
        dE = abs(o["energy"][b] - ref.energy) / n
        dF = np.abs(F - ref.forces)
        vol = abs(np.linalg.det(structs[b].cell))
        dW = np.abs(o["virial"][b] - ref.virial).max() / vol
        print(f"[batch {prec}] struct {b} n={n} edges={ref.n_edges}: dE/N={dE:.2e} max|dF|={dF.max():.2e} "
              f"|dW|/V={dW:.2e}")
        if prec == "fp32":
            assert dE <= 1e-6 and dF.max() <= 1e-4 and dF.max() <= 1e-5 * max(np.abs(ref.forces).max(), 1e-3)
            assert dW <= 1e-8
        else:
            rms = np.sqrt(np.mean(dF ** 2))
            assert dE <= 1e-3 and rms <= 5e-3 and rms <= 2e-2 * max(np.sqrt(np.mean(ref.forces ** 2)), 1e-3)
            assert dW <= 1e-5


def test_batch_invariants(batch_case):
    structs, batch, out, refs = batch_case
    o = out["fp32"]
    for b in range(batch.B):
        a0, a1 = batch.atom_ptr[b], batch.atom_ptr[b + 1]
        assert np.abs(o["forces"][a0:a1].sum(axis=0)).max() <= 1e-6
        Wv = o["virial"][b]
        assert np.abs(Wv - Wv.T).max() <= 1e-6 * max(1.0, np.abs(Wv).max())
    assert out["fp32"]["n_edges"] == out["bf16"]["n_edges"]
