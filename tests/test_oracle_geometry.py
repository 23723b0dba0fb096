"""Pins of the oracle's neighbour search, radial basis, harmonics and
coupling tensors against library routines, closed forms and invariants."""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.special import eval_legendre

import oracle
import workloads as W
from oracle.gaunt import coupling_tensor, gaunt_tensor, layer_paths, natural
from oracle.neighbors import neighbor_list

RC = 5.0


# ------------------------------------------------------------------ neighbours

def _pairs(i, j):
    return set(zip(np.minimum(i, j).tolist(), np.maximum(i, j).tolist()))


@pytest.mark.parametrize("n,L,seed", [(128, 11.5, 1), (900, 22.0, 2)])
def test_neighbors_match_ckdtree(n, L, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (n, 3))
    i, j, S = neighbor_list(pos, np.diag([L] * 3), [True] * 3, RC)
    tree = cKDTree(pos, boxsize=L)
    ref = tree.query_pairs(RC, output_type="ndarray")
    assert i.size == 2 * len(ref)
    assert _pairs(i, j) == set(map(tuple, ref.tolist()))


def test_small_workload_matches_ckdtree():
    s = W.small_system()
    i, j, S = neighbor_list(s.positions, s.cell, s.pbc, RC)
    ref = cKDTree(np.mod(s.positions, 11.5), boxsize=11.5).query_pairs(RC, output_type="ndarray")
    assert i.size == 2 * len(ref)
    assert _pairs(i, j) == set(map(tuple, ref.tolist()))


def test_perfect_lattice_has_32_neighbours():
    # shells a, a*sqrt2, a*sqrt3, 2a (6+12+8+6); a*sqrt5 = 5.086 A is outside
    pos = W.lattice_positions(6, 6, 6, W.LATTICE_A, 0, jitter=0.0)
    i, j, S = neighbor_list(pos, np.diag([6 * W.LATTICE_A] * 3), [True] * 3, RC)
    assert np.all(np.bincount(i, minlength=216) == 32)


def test_one_atom_thin_cell_image_loop():
    # a single atom in a 2.274 A cube: all 32 lattice images within 5 A
    a = W.LATTICE_A
    i, j, S = neighbor_list(np.zeros((1, 3)), np.diag([a] * 3), [True] * 3, RC)
    assert i.size == 32
    n2 = np.sum(S * S, axis=1)
    assert sorted(np.bincount(n2)[1:].tolist()) == sorted([6, 12, 8, 6])


def test_triclinic_basis_of_same_lattice():
    a = W.LATTICE_A
    pos = W.lattice_positions(3, 3, 3, a, 0, jitter=0.0)
    cell = np.array([[3 * a, 0, 0], [3 * a, 3 * a, 0], [0, 0, 3 * a]])   # sheared basis, same lattice
    i, j, S = neighbor_list(pos, cell, [True] * 3, RC)
    assert np.all(np.bincount(i, minlength=27) == 32)


def test_edge_symmetry_and_nonperiodic_axis():
    s = W.slab_full_system(12, 5, 5, 7, 8)
    pbc = np.array([False, True, True])
    i, j, S = neighbor_list(s.positions, s.cell, pbc, RC)
    fwd = set(zip(i.tolist(), j.tolist(), map(tuple, S.tolist())))
    rev = set(zip(j.tolist(), i.tolist(), map(tuple, (-S).tolist())))
    assert fwd == rev
    assert np.all(S[:, 0] == 0)
    r = oracle.edge_vectors(s.positions, s.cell, i, j, S)
    assert np.all(np.sum(r * r, axis=1) < RC * RC)


# ------------------------------------------------------------------ radial

def test_envelope_closed_form():
    f, df = oracle.envelope(np.array([0.0, 2.5, 5.0 - 1e-9]), RC, 6)
    assert f[0] == 1.0 and df[0] == 0.0
    x = 0.5
    assert f[1] == pytest.approx(1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8, abs=1e-15)
    assert abs(f[2]) < 1e-12 and abs(df[2]) < 1e-9
    # f is the polynomial 1 - 28x^6 + 48x^7 - 21x^8 inside the cutoff, and
    # that polynomial has f(1) = f'(1) = f''(1) = 0
    poly = np.polynomial.Polynomial([1, 0, 0, 0, 0, 0, -28, 48, -21])
    for k in range(3):
        assert poly.deriv(k)(1.0) == pytest.approx(0.0, abs=1e-12)
    xs = np.linspace(0.05, 0.95, 7)
    f, df = oracle.envelope(xs * RC, RC, 6)
    assert np.allclose(f, poly(xs), atol=1e-14)
    assert np.allclose(df, poly.deriv(1)(xs) / RC, atol=1e-13)


def test_bessel_limit_and_derivatives():
    n = np.arange(1, 9)
    B, _ = oracle.bessel_basis(np.array([1e-7]), RC, 8)
    assert np.allclose(B[0], math.sqrt(2 / RC) * n * math.pi / RC, rtol=1e-10)
    d = np.linspace(0.7, 4.9, 11)
    e, de = oracle.radial_features(d, RC, 8, 6)
    h = 1e-6
    ep, _ = oracle.radial_features(d + h, RC, 8, 6)
    em, _ = oracle.radial_features(d - h, RC, 8, 6)
    assert np.allclose(de, (ep - em) / (2 * h), atol=1e-7)


# ------------------------------------------------------------------ harmonics

def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_sh_norm_and_z_axis():
    rng = np.random.default_rng(0)
    Y = oracle.real_sh(_unit(rng, 50))
    for l in range(3):
        assert np.allclose(np.sum(Y[:, l * l:(l + 1) ** 2] ** 2, axis=1), 2 * l + 1)
    Yz = oracle.real_sh(np.array([[0.0, 0.0, 1.0]]))[0]
    assert np.allclose(Yz, [1, 0, math.sqrt(3), 0, 0, 0, math.sqrt(5), 0, 0])


def test_sh_addition_theorem():
    # sum_m Y_lm(u) Y_lm(v) = (2l+1) P_l(u.v) for component-normalised harmonics
    rng = np.random.default_rng(1)
    u, v = _unit(rng, 40), _unit(rng, 40)
    Yu, Yv = oracle.real_sh(u), oracle.real_sh(v)
    c = np.sum(u * v, axis=1)
    for l in range(3):
        b = slice(l * l, (l + 1) ** 2)
        assert np.allclose(np.sum(Yu[:, b] * Yv[:, b], axis=1), (2 * l + 1) * eval_legendre(l, c))


def test_sh_equivariance_and_parity():
    rng = np.random.default_rng(2)
    u = _unit(rng, 60)
    Q = _rotation(rng)
    Y, YQ = oracle.real_sh(u), oracle.real_sh(u @ Q.T)
    for l in range(3):
        b = slice(l * l, (l + 1) ** 2)
        D, *_ = np.linalg.lstsq(Y[:, b], YQ[:, b], rcond=None)
        assert np.allclose(Y[:, b] @ D, YQ[:, b], atol=1e-12)
        assert np.allclose(D.T @ D, np.eye(2 * l + 1), atol=1e-12)
        assert np.allclose(oracle.real_sh(-u)[:, b], (-1) ** l * Y[:, b])


def test_sh_gradient_fd():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((7, 3))
    G = oracle.real_sh_grad(u)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3); e[k] = h
        fd = (oracle.real_sh(u + e) - oracle.real_sh(u - e)) / (2 * h)
        assert np.allclose(G[:, :, k], fd, atol=1e-8)


# ------------------------------------------------------------------ coupling

ALL = [(a, b, c) for a in range(3) for b in range(3) for c in range(3) if natural(a, b, c)]


def test_path_counts_and_nnz():
    assert len(ALL) == 11
    nnz = [int(np.sum(np.abs(coupling_tensor(*p)) > 1e-12)) for p in
           [(0, 0, 0), (0, 1, 1), (0, 2, 2), (1, 0, 1), (1, 1, 0), (1, 1, 2),
            (1, 2, 1), (2, 0, 2), (2, 1, 1), (2, 2, 0), (2, 2, 2)]]
    assert nnz == [1, 3, 5, 3, 3, 11, 11, 5, 11, 5, 25]
    assert layer_paths(1, 2) == [(0, 0, 0), (0, 1, 1), (0, 2, 2)]
    assert len(layer_paths(2, 2)) == 11 and len(layer_paths(2, 1)) == 4


def test_coupling_special_cases():
    for l in range(3):
        I = np.eye(2 * l + 1) / math.sqrt(2 * l + 1)
        assert np.allclose(coupling_tensor(0, l, l)[0], I)
        assert np.allclose(coupling_tensor(l, 0, l)[:, 0, :], I)
        assert np.allclose(coupling_tensor(l, l, 0)[:, :, 0], I)


@pytest.mark.parametrize("p", ALL)
def test_coupling_equivariance_norm_sign(p):
    rng = np.random.default_rng(4)
    Q = _rotation(rng)
    u = _unit(rng, 80)
    Y, YQ = oracle.real_sh(u), oracle.real_sh(u @ Q.T)
    D = []
    for l in range(3):
        b = slice(l * l, (l + 1) ** 2)
        D.append(np.linalg.lstsq(Y[:, b], YQ[:, b], rcond=None)[0].T)   # YQ = D Y
    Cp = coupling_tensor(*p)
    x, y = rng.standard_normal(2 * p[0] + 1), rng.standard_normal(2 * p[1] + 1)
    lhs = np.einsum("abk,a,b->k", Cp, D[p[0]] @ x, D[p[1]] @ y)
    rhs = D[p[2]] @ np.einsum("abk,a,b->k", Cp, x, y)
    assert np.allclose(lhs, rhs, atol=1e-12)
    assert np.linalg.norm(Cp) == pytest.approx(1.0, abs=1e-14)
    # sign: the full contraction with Y(v) three times is a positive constant
    v = _unit(rng, 5)
    Yv = oracle.real_sh(v)
    b = [slice(l * l, (l + 1) ** 2) for l in p]
    val = np.einsum("abk,ea,eb,ek->e", Cp, Yv[:, b[0]], Yv[:, b[1]], Yv[:, b[2]])
    assert np.all(val > 0) and np.allclose(val, val[0])


def test_quadrature_is_converged():
    # the integrand has degree <= 6, so the 8 x 16 product rule is exact:
    # a 24 x 50 product rule and a fine midpoint rule must agree with it
    def product_rule(nz, nph):
        zs, wz = np.polynomial.legendre.leggauss(nz)
        ph = 2 * np.pi * np.arange(nph) / nph
        Z, P = np.meshgrid(zs, ph, indexing="ij")
        st = np.sqrt(1 - Z * Z)
        u = np.stack([st * np.cos(P), st * np.sin(P), Z], -1).reshape(-1, 3)
        return u, (np.repeat(wz[:, None], nph, 1) * 2 * np.pi / nph).reshape(-1)

    nt = nph = 300
    th = (np.arange(nt) + 0.5) * np.pi / nt
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    um = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    wm = (np.sin(T) * (np.pi / nt) * (2 * np.pi / nph)).reshape(-1)
    for u, w, tol in [(*product_rule(24, 50), 1e-12), (um, wm, 2e-3)]:
        Y = oracle.real_sh(u)
        for p in ALL:
            b = [slice(l * l, (l + 1) ** 2) for l in p]
            G = np.einsum("q,qa,qb,qc->abc", w, Y[:, b[0]], Y[:, b[1]], Y[:, b[2]])
            assert np.allclose(G, gaunt_tensor(*p), atol=tol)
