"""Pins of the oracle's MD integrator (CPU).

* Philox4x32-10 against the known-answer vectors published with the
  generator (Salmon et al., SC'11, Random123 distribution): counter 0 /
  key 0, all-ones counter and key, and the pi-digit counter and key.
* Box-Muller normals: sample mean and variance.
* Velocity Verlet on a harmonic force F = -k x has the closed form
  x_n = cos(n theta) with cos(theta) = 1 - (omega dt)^2 / 2 (x_0 = 1, v_0 = 0):
  pins the order and the dt/2 factors of the B and A steps and the unit
  factor (omega^2 = factor * k / m).
* Free flight (no neighbours within the cutoff): x_n = x_0 + n dt v_0 exactly.
* Time reversibility of velocity Verlet with the model's forces: n steps,
  negated velocities, n steps return to the start.
* Second order: the energy error of velocity Verlet over a fixed time
  shrinks by about 4 when dt halves.
* Langevin O step: with zero forces the velocity variance relaxes to
  kB T / m (equipartition).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import md

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert md.philox4x32_10(ctr, key) == want


def test_box_muller_moments():
    z = np.concatenate([md.normals3(12345, a, 3) for a in range(6000)])
    assert abs(z.mean()) < 0.03
    assert abs(z.var() - 1.0) < 0.05


def test_harmonic_closed_form():
    k, m, dt, n = 2.0, 1.5, 0.7, 40
    omega2 = md.ACCEL * k / m
    h2 = omega2 * dt * dt
    theta = math.acos(1.0 - h2 / 2.0)
    x0 = np.array([[1.0, 0.0, 0.0]])
    tr = md.run(x0, np.zeros((1, 3)), np.array([0]), [m], None, None, None, None, None, dt, n,
                force_fn=lambda x: (0.5 * k * float(np.sum(x * x)), -k * x))
    xs = tr.positions[:, 0, 0]
    assert np.allclose(xs, np.cos(np.arange(n + 1) * theta), atol=1e-12)


def _cluster(n=8, seed=5):
    """A few atoms inside one cutoff sphere in a large non-periodic box."""
    rng = np.random.default_rng(seed)
    pos = 20.0 + rng.uniform(-2.2, 2.2, size=(n, 3))
    sp = rng.integers(0, 2, size=n).astype(np.int32)
    return pos, sp, np.diag([40.0, 40.0, 40.0]), np.array([False, False, False])


def test_free_flight_exact():
    pos = np.array([[5.0, 5.0, 5.0], [25.0, 25.0, 25.0]])
    v = np.array([[0.01, -0.02, 0.03], [-0.01, 0.0, 0.02]])
    hp = W.HP_SMALL
    blob = W.make_weights(hp, 103)
    tr = md.run(pos, v, np.array([0, 1]), [6.94, 15.999], np.diag([40.0] * 3), np.array([False] * 3), blob, hp,
                2, dt=0.5, n_steps=6)
    for s in range(7):
        assert np.allclose(tr.positions[s], pos + s * 0.5 * v, atol=1e-12, rtol=0)
        assert np.array_equal(tr.velocities[s], v)


def test_velocity_verlet_reversible():
    pos, sp, cell, pbc = _cluster()
    hp = W.HP_SMALL
    blob = W.make_weights(hp, 103)
    v0 = W.velocities(len(pos), 0.02, 11)
    a = md.run(pos, v0, sp, [6.94, 15.999], cell, pbc, blob, hp, 2, dt=1.0, n_steps=8)
    b = md.run(a.positions[-1], -a.velocities[-1], sp, [6.94, 15.999], cell, pbc, blob, hp, 2, dt=1.0, n_steps=8)
    assert np.abs(b.positions[-1] - pos).max() < 1e-9
    assert np.abs(b.velocities[-1] + v0).max() < 1e-9


def test_energy_error_second_order():
    pos, sp, cell, pbc = _cluster(n=6, seed=9)
    hp = W.HP_SMALL
    blob = W.make_weights(hp, 103)
    v0 = W.velocities(len(pos), 0.05, 12)
    masses = [6.94, 15.999]

    def drift(dt, n):
        tr = md.run(pos, v0, sp, masses, cell, pbc, blob, hp, 2, dt=dt, n_steps=n)
        m = np.asarray(masses)[sp]
        e0 = md.evaluate(pos, sp, cell, pbc, blob, hp, K=2).energy + md.kinetic_energy(v0, m)
        return np.abs(tr.epot + tr.ekin - e0).max()

    d1, d2 = drift(2.0, 10), drift(1.0, 20)
    assert d1 > 0 and 3.0 < d1 / d2 < 5.0


def test_langevin_equipartition():
    n, masses, T, gamma, dt = 200, [6.94, 30.973762, 15.999], 300.0, 0.1, 1.0
    sp = (np.arange(n) % 3).astype(np.int32)
    tr = md.run(np.zeros((n, 3)), np.zeros((n, 3)), sp, masses, None, None, None, None, None, dt, 60,
                friction=gamma, temperature=T, seed=2024, force_fn=lambda x: (0.0, np.zeros_like(x)))
    m = np.asarray(masses)[sp]
    kT = md.BOLTZMANN_EV * T
    ratio = (m[:, None] * tr.velocities[-1] ** 2 / md.ACCEL).mean() / kT
    assert 0.85 < ratio < 1.15


def test_accel_unit_factor_from_faraday_constant():
    """The force/mass -> acceleration factor, pinned by a value the code does
    not derive it from: e/u equals the Faraday constant over the molar mass
    constant, F = 96485.33212 C/mol (CODATA 2018) and M_u = 1e-3 kg/mol (to
    4e-10 relative), so 1 eV/(A amu) = F / M_u * 1e10 m/s^2, and
    1 m/s^2 = 1e-20 A/fs^2; the textbook form of the same fact is
    1 amu A^2/fs^2 = 103.6427 eV."""
    faraday, molar_mass_const = 96485.33212, 1e-3
    want = faraday / molar_mass_const * 1e10 * 1e-20
    assert md.ACCEL == pytest.approx(want, rel=1e-9)
    assert md.ACCEL == pytest.approx(9.648533e-3, rel=1e-6)
    assert 1.0 / md.ACCEL == pytest.approx(103.6427, rel=1e-6)
