"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (per atom for the energy, eV and Angstrom):
  FP32 form: |dE|/N <= 1e-6, max |dF| <= 1e-4, and relative to the oracle's
             force scale max |dF| <= 1e-5 * max|F| (FP32 rounding over a few
             thousand operations per output);
  BF16 form: |dE|/N <= 1e-3, RMS dF <= 5e-3, and RMS dF <= 2e-2 * RMS F
             (BF16 keeps 8 mantissa bits: ~0.4 % per rounding, averaged over
             the 64-wide hidden layer and the ~40 edges of a row).
The virial W = -sum_e r_e (x) g_e is a sum of large terms of both signs, so
its relative error is about ten times the force error; it is bounded as a
stress, |dW|/V <= 1e-8 eV/A^3 (FP32) and 1e-5 eV/A^3 = 1.6 MPa (BF16), and
its relative error is printed.  The edge list must be identical as a set of
(i, j, S) triples.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


@pytest.fixture(scope="module")
def M():
    import paper_2509_21694_amd as mod
    return mod


def dev_inputs(torch, s):
    pos = torch.tensor(np.ascontiguousarray(s.positions), dtype=torch.float64, device="cuda")
    sp = torch.tensor(np.ascontiguousarray(s.species), dtype=torch.int32, device="cuda")
    return pos, sp


def edge_set(i, j, S):
    return set(zip(np.asarray(i).tolist(), np.asarray(j).tolist(), map(tuple, np.asarray(S).tolist())))


def compare(o, ref, n, prec, label, volume, n_owned=None):
    E = float(o["energy"].cpu()[0])
    F = o["forces"].cpu().numpy()
    Wv = o["virial"].cpu().numpy()
    dE = abs(E - ref.energy) / n
    dF = np.abs(F - ref.forces)
    fmax, frms = np.abs(ref.forces).max(), np.sqrt(np.mean(ref.forces ** 2))
    rms = np.sqrt(np.mean(dF ** 2))
    dW = np.abs(Wv - ref.virial).max()
    print(f"[{label}] {prec}: dE/N={dE:.3e} max|dF|={dF.max():.3e} rms dF={rms:.3e} "
          f"(|F|max={fmax:.3e} rms={frms:.3e}) max|dW|={dW:.3e} (|W|max={np.abs(ref.virial).max():.3e}, "
          f"|dW|/V={dW / volume:.3e} eV/A^3)")
    if prec == "fp32":
        assert dE <= 1e-6
        assert dF.max() <= 1e-4
        assert dF.max() <= 1e-5 * fmax
        assert dW / volume <= 1e-8
    else:
        assert dE <= 1e-3
        assert rms <= 5e-3
        assert rms <= 2e-2 * frms
        assert dW / volume <= 1e-5
    if o.get("atom_energy") is not None:
        # a partition share (n_owned < N) is trimmed to the roots' receptive
        # field: atom energies on the roots, zero elsewhere
        ae = o["atom_energy"].cpu().numpy()
        k = ae.shape[0] if n_owned is None else n_owned
        tol = 1e-6 if prec == "fp32" else 1e-3
        assert np.abs(ae[:k] - ref.atom_energy[:k]).max() <= tol
        assert np.all(ae[k:] == 0.0)


# ----------------------------------------------------------- neighbour list

NBR_CASES = ["small", "mpdp", "slab_pbc011", "thin_cell", "unwrapped", "cluster", "dense", "three_bins", "cutoff_shell"]


def nbr_case(name):
    if name == "small":
        s = W.small_system()
        return s.positions, s.cell, s.pbc
    if name == "mpdp":
        s = W.mpdp_system()
        return s.positions, s.cell, s.pbc
    if name == "slab_pbc011":
        s = W.slab_full_system(60, 10, 10, 3, 4)
        return s.positions, s.cell, np.array([False, True, True])
    if name == "thin_cell":
        rng = np.random.default_rng(5)
        cell = np.diag([4.1, 6.3, 9.7])
        return rng.uniform(0, 1, (6, 3)) * np.diag(cell), cell, np.array([True, True, True])
    if name == "unwrapped":
        s = W.small_system()
        rng = np.random.default_rng(6)
        shift = rng.integers(-3, 4, (128, 3)) * 11.5
        return s.positions + shift, s.cell, s.pbc
    if name == "cluster":
        rng = np.random.default_rng(7)
        return rng.uniform(0, 14, (300, 3)), np.eye(3) * 14, np.array([False, False, False])
    if name == "dense":
        # 0.41 atoms/A^3: about 1,700 candidates per atom in the 27 bins, more
        # than the counting pass keeps masks for, so the fill tests them again
        a = 1.35
        pos = W.lattice_positions(12, 12, 12, a, 8, jitter=0.05)
        return pos, np.eye(3) * 12 * a, np.array([True, True, True])
    if name == "three_bins":
        # 0.15 atoms/A^3 in three 5 A bins per direction: about 500 candidates
        # per atom (on both sides of the kept-mask limit) and about 78
        # neighbours, more than one 64-lane round of the fill
        a = 1.8825
        pos = W.lattice_positions(8, 8, 8, a, 9, jitter=0.1)
        return pos, np.eye(3) * 8 * a, np.array([True, True, True])
    if name == "cutoff_shell":
        # 2.5 A lattice in a 20 A box (three stencil bins per axis): the shell
        # at 2a = r_cut is jittered by 1e-7 A, so thousands of pairs lie far
        # inside the FP32 prefilter's band and are decided by the FP64 test
        a = 2.5
        pos = W.lattice_positions(8, 8, 8, a, 10, jitter=1e-7)
        return pos, np.eye(3) * 8 * a, np.array([True, True, True])
    raise KeyError(name)


@pytest.mark.parametrize("name", NBR_CASES)
def test_neighbor_list_bit_exact(torch, M, name):
    pos, cell, pbc = nbr_case(name)
    ri, rj, rS = oracle.neighbor_list(pos, cell, pbc, 5.0)
    p = torch.tensor(pos, dtype=torch.float64, device="cuda")
    gi, gj, gS = M.neighbor_list(p, cell, pbc, 5.0)
    got = edge_set(gi.cpu().numpy(), gj.cpu().numpy(), gS.cpu().numpy())
    ref = edge_set(ri, rj, rS)
    print(f"[{name}] edges gpu={len(got)} oracle={len(ref)}")
    assert gi.numel() == ri.size
    assert got == ref


# ----------------------------------------------------------- small system

@pytest.fixture(scope="module")
def small_case():
    s = W.small_system()
    blob = W.make_weights(W.HP_SMALL, W.WEIGHT_SEEDS["small"])
    refs = {K: oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, W.HP_SMALL, K=K) for K in (1, 2)}
    return s, blob, refs


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("K", [2, 1])
def test_small_parity(torch, M, small_case, prec, K):
    s, blob, refs = small_case
    model = M.Model(W.HP_SMALL, blob)
    pos, sp = dev_inputs(torch, s)
    o = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision=prec, atom_energy=True)
    assert o["n_edges"] == refs[K].n_edges
    compare(o, refs[K], s.n_atoms, prec, f"small K={K}", abs(np.linalg.det(s.cell)))


def test_small_e0_and_ghost_rows(torch, M):
    """Per-species offsets and a partition-style evaluation (root atoms
    first, ghosts contribute no energy but receive partial forces)."""
    s = W.small_system()
    blob = W.make_weights(W.HP_SMALL, 9, e0=[0.7, -1.3])
    n_own = 50
    ref = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, W.HP_SMALL, n_owned=n_own)
    model = M.Model(W.HP_SMALL, blob)
    pos, sp = dev_inputs(torch, s)
    o = model.evaluate(pos, sp, s.cell, s.pbc, precision="fp32", n_owned=n_own, atom_energy=True)
    compare(o, ref, s.n_atoms, "fp32", "small n_owned=50", abs(np.linalg.det(s.cell)), n_owned=n_own)


def test_determinism_and_autograd(torch, M, small_case):
    s, blob, refs = small_case
    model = M.Model(W.HP_SMALL, blob)
    pos, sp = dev_inputs(torch, s)
    a = model.evaluate(pos, sp, s.cell, s.pbc, precision="bf16")
    b = model.evaluate(pos, sp, s.cell, s.pbc, precision="bf16")
    assert torch.equal(a["forces"], b["forces"]) and torch.equal(a["energy"], b["energy"])
    assert torch.equal(a["virial"], b["virial"])
    x = pos.clone().requires_grad_(True)
    E, Wv = M.energy(x, model, sp, s.cell, s.pbc, precision="fp32")
    E.backward()
    assert np.allclose(-x.grad.cpu().numpy(), refs[2].forces, atol=1e-5)
    assert abs(float(E.detach()) - refs[2].energy) / 128 <= 1e-6


def test_data_errors_reported(torch, M, small_case):
    s, blob, _ = small_case
    model = M.Model(W.HP_SMALL, blob)
    pos, sp = dev_inputs(torch, s)
    bad = sp.clone()
    bad[3] = 7
    with pytest.raises(M.MpipError) as e:
        model.evaluate(pos, bad, s.cell, s.pbc)
    assert e.value.status == M.EINVAL
    p2 = pos.clone()
    p2[5] = p2[9]
    with pytest.raises(M.MpipError) as e:
        model.evaluate(p2, sp, s.cell, s.pbc)
    assert e.value.status == M.EINVAL
    # too small an edge capacity is reported and retried with the exact count
    o = model.evaluate(pos, sp, s.cell, s.pbc, max_edges=100)
    assert o["n_edges"] == 6016


# ----------------------------------------------------------- depth pruning

@pytest.mark.parametrize("K", [2, 6])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mpdp_parity(torch, M, K, prec):
    path = os.path.join(GOLDEN, f"mpdp_K{K}.npz")
    if not os.path.exists(path):
        pytest.skip("golden file missing (tests/golden/make_golden.py)")
    g = np.load(path)

    class R:
        energy = float(g["energy"])
        forces = g["forces"]
        virial = g["virial"]
        atom_energy = g["atom_energy"]

    s = W.mpdp_system()
    model = M.Model(W.HP_MPDP, W.make_weights(W.HP_MPDP, W.WEIGHT_SEEDS["mpdp"]))
    pos, sp = dev_inputs(torch, s)
    o = model.evaluate(pos, sp, s.cell, s.pbc, K=K, precision=prec, atom_energy=True)
    assert o["n_edges"] == int(g["n_edges"])
    compare(o, R, s.n_atoms, prec, f"mpdp K={K}", abs(np.linalg.det(s.cell)))


# ----------------------------------------------------------- specialised kernels

FAST_CASES = [(2, 64, 3), (1, 128, 3), (2, 128, 3), (1, 64, 8)]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("L,C,S", FAST_CASES)
def test_fast_kernels_parity(torch, M, L, C, S, prec):
    """First / last layer specialised kernels (64 and 128 channels) against
    the oracle on the 128-atom box, and against the generic kernels."""
    import os as _os
    s = W.small_system()
    hp = W.HParams(n_species=S, n_layers=2, l_max=L, channels=C)
    sp_np = (np.arange(128) * 7 % S).astype(np.int32)
    blob = W.make_weights(hp, 40 + L + C + S)
    ref = oracle.evaluate(s.positions, sp_np, s.cell, s.pbc, blob, hp)
    model = M.Model(hp, blob)
    _os.environ["MPIP_FORCE_GENERIC"] = "1"
    try:
        generic = M.Model(hp, blob)
    finally:
        del _os.environ["MPIP_FORCE_GENERIC"]
    pos = torch.tensor(s.positions, dtype=torch.float64, device="cuda")
    sp = torch.tensor(sp_np, dtype=torch.int32, device="cuda")
    o = model.evaluate(pos, sp, s.cell, s.pbc, precision=prec, atom_energy=True)
    og = generic.evaluate(pos, sp, s.cell, s.pbc, precision=prec, atom_energy=True)
    compare(o, ref, 128, prec, f"fast L={L} C={C} S={S}", abs(np.linalg.det(s.cell)))
    compare(og, ref, 128, prec, f"generic L={L} C={C} S={S}", abs(np.linalg.det(s.cell)))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_edge_length_range_parity(torch, M, prec):
    """The specialised kernels (K = 2, l_max = 2, C = 128) over the whole
    range of edge lengths, against the oracle: isolated triangles, 20 A
    apart in a non-periodic box, whose sides run from 0.4 A to a hair under
    r_c, so the BF16 form's radial table is read in its first and last
    intervals (tau near 0 and near 1) as well as in between."""
    hp = W.HParams(n_species=3, n_layers=2, l_max=2, channels=128)
    rng = np.random.default_rng(17)
    firsts = [0.4, 0.9, 1.7, 2.6, 3.5, 4.2, 4.8, 4.99, 4.9999, hp.r_cut * (1.0 - 1e-7)]
    pos = []
    for t, d1 in enumerate(firsts):
        c = np.array([20.0 * (t % 5), 20.0 * (t // 5), 0.0]) + 10.0
        u1, u2 = rng.standard_normal(3), rng.standard_normal(3)
        d2 = firsts[(t + 3) % len(firsts)]
        pos += [c, c + d1 * u1 / np.linalg.norm(u1), c + d2 * u2 / np.linalg.norm(u2)]
    pos = np.array(pos)
    n = pos.shape[0]
    cell = np.diag([120.0, 60.0, 40.0])
    pbc = (False, False, False)
    sp_np = (np.arange(n) % 3).astype(np.int32)
    blob = W.make_weights(hp, 77)
    ref = oracle.evaluate(pos, sp_np, cell, pbc, blob, hp)
    model = M.Model(hp, blob)
    o = model.evaluate(torch.tensor(pos, dtype=torch.float64, device="cuda"),
                       torch.tensor(sp_np, dtype=torch.int32, device="cuda"), cell, pbc, precision=prec,
                       atom_energy=True)
    assert o["n_edges"] == 2 * sum(1 for t in range(len(firsts)) for (a, b) in ((0, 1), (0, 2), (1, 2))
                                   if np.linalg.norm(pos[3 * t + a] - pos[3 * t + b]) < hp.r_cut)
    compare(o, ref, n, prec, "edge-length range", float(np.linalg.det(cell)))
