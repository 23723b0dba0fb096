"""GPU parity of the on-device MD driver (mpip_md_run) against the oracle's
BAOAB / velocity-Verlet integrator with FP64 forces.

The skin variant (neighbour list of radius r_c + skin reused while atoms
move less than skin/2) selects the same edges as a rebuild, so it is held
to the same bounds against the oracle, with atoms fast enough to force a
rebuild inside the run; the energy-conservation runs use it too.

Tolerances: over a few steps the trajectory differs from the oracle's by
the force error (FP32 form: <= 1e-4 eV/A) times dt^2/m, so positions agree
to 1e-6 A and velocities to 1e-6 A/fs; the per-step potential energy as in
the single-evaluation parity (|dE|/N <= 1e-6 eV) and the kinetic energy to
1e-6 relative.  The Langevin noise is the same Philox4x32-10 sequence on
both sides (integer arithmetic), so stochastic trajectories are compared
the same way.  Energy conservation (velocity Verlet, 60 steps of 1 fs,
4096 atoms): FP32 form |dE_total|/N <= 1e-5 eV; BF16 form (its forces are
not the exact gradient of its rounded energy) <= 1e-3 eV, the BF16 energy
tolerance.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import md as omd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


@pytest.fixture(scope="module")
def M():
    import paper_2509_21694_amd as mod
    return mod


def _run_both(torch, M, friction, temperature, seed, n_steps=6, dt=0.5, skin=0.0, sigma=0.02):
    s = W.small_system()
    hp = W.HP_SMALL
    blob = W.make_weights(hp, 103)
    masses = [6.94, 15.999]
    v0 = W.velocities(s.n_atoms, sigma, 31)
    ref = omd.run(s.positions, v0, s.species, masses, s.cell, s.pbc, blob, hp, 2, dt=dt, n_steps=n_steps,
                  friction=friction, temperature=temperature, seed=seed)
    model = M.Model(hp, blob)
    x = torch.tensor(s.positions, dtype=torch.float64, device="cuda").contiguous()
    v = torch.tensor(v0, dtype=torch.float64, device="cuda").contiguous()
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    ms = torch.tensor(masses, dtype=torch.float64, device="cuda")
    print(f"[md] small system, {n_steps} steps, friction {friction}, skin {skin}", flush=True)
    ep, ek, F = model.md_run(x, v, sp, ms, s.cell, s.pbc, dt=dt, n_steps=n_steps, friction=friction,
                             temperature=temperature, seed=seed, skin=skin, K=2, precision="fp32")
    torch.cuda.synchronize()
    return s, ref, x.cpu().numpy(), v.cpu().numpy(), F.cpu().numpy(), ep.cpu().numpy(), ek.cpu().numpy()


def _check(s, ref, x, v, F, ep, ek):
    n = s.n_atoms
    dx = np.abs(x - ref.positions[-1]).max()
    dv = np.abs(v - ref.velocities[-1]).max()
    dF = np.abs(F - ref.forces[-1]).max()
    dEp = np.abs(ep - ref.epot).max() / n
    dEk = np.abs(ek - ref.ekin).max() / np.abs(ref.ekin).max()
    print(f"[md] max|dx|={dx:.2e} max|dv|={dv:.2e} max|dF|={dF:.2e} dEpot/N={dEp:.2e} dEkin rel={dEk:.2e}")
    assert dx <= 1e-6 and dv <= 1e-6 and dF <= 1e-4 and dEp <= 1e-6 and dEk <= 1e-6


def test_md_velocity_verlet_matches_oracle(torch, M):
    _check(*_run_both(torch, M, 0.0, 0.0, 0))


def test_md_langevin_matches_oracle(torch, M):
    _check(*_run_both(torch, M, 0.05, 300.0, 77))


def test_md_skin_list_matches_oracle(torch, M):
    # fast atoms (0.05 A/fs, 12 steps of 1 fs) so that the list of radius
    # r_c + 0.8 A is rebuilt during the run and reused in between
    _check(*_run_both(torch, M, 0.0, 0.0, 0, n_steps=12, dt=1.0, skin=0.8, sigma=0.05))


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-5), ("bf16", 1e-3)])
def test_md_energy_conservation(torch, M, prec, bound):
    s = W.bulk_system(16, 601, 602)
    hp = W.HP_BATCH
    blob = W.make_weights(hp, 603)
    model = M.Model(hp, blob)
    x = torch.tensor(s.positions, dtype=torch.float64, device="cuda").contiguous()
    v = torch.tensor(W.velocities(s.n_atoms, 0.01, 604), dtype=torch.float64, device="cuda").contiguous()
    sp = torch.tensor(s.species, dtype=torch.int32, device="cuda")
    ms = torch.tensor(W.MASSES_LPO, dtype=torch.float64, device="cuda")
    e0 = model.evaluate(x, sp, s.cell, s.pbc, K=2, precision=prec)
    m = np.asarray(W.MASSES_LPO)[s.species]
    etot0 = float(e0["energy"].cpu()[0]) + omd.kinetic_energy(v.cpu().numpy(), m)
    print(f"[md] 4096 atoms, {prec}, 60 steps", flush=True)
    ep, ek, _ = model.md_run(x, v, sp, ms, s.cell, s.pbc, dt=1.0, n_steps=60, forces=e0["forces"], K=2,
                             precision=prec, skin=0.5)
    etot = ep.cpu().numpy() + ek.cpu().numpy()
    drift = np.abs(etot - etot0).max() / s.n_atoms
    print(f"[md] {prec}: max |E_total - E_total(0)| / N = {drift:.3e} eV (kinetic {float(ek[-1]) / s.n_atoms:.3e})")
    assert drift <= bound
