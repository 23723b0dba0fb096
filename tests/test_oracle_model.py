"""Pins of the oracle's energy, forces and virial.

The potential has no printed worked example, so the oracle is pinned by
(a) an independent closed form of the K = 1 and K = 2 models written with
Legendre polynomials of bond angles (no spherical harmonics, no coupling
tables, no shared parser), (b) finite differences of the energy for forces
and virial, (c) invariances and equivariances, (d) special cases (dimer,
separability, depth-pruning truncation), and (e) the partition rules of
Methods "Graph Partitioning" / "Global Output Integration".
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

RC = 5.0


def hp_of(L, C, T, S=3):
    return W.HParams(n_species=S, n_layers=T, l_max=L, channels=C)


def cluster(n, seed, box=9.0, dmin=1.6):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, box, 3)
        if all(np.linalg.norm(p - q) > dmin for q in pts):
            pts.append(p)
    return np.array(pts), rng.integers(0, 3, n).astype(np.int32)


def ev(pos, sp, hp, blob, K=None, cell=None, pbc=(False,) * 3, **kw):
    cell = np.eye(3) * 100.0 if cell is None else cell
    return oracle.evaluate(pos, sp, cell, np.array(pbc), blob, hp, K=K, **kw)


# ------------------------------------------------------------- closed forms

def _unpack(blob, hp):
    """The test's own reading of the blob, driven by the generator's layout."""
    out, off = {}, 0
    for name, shape, _ in W.weight_layout(hp):
        n = int(np.prod(shape))
        out[name] = blob[off:off + n].astype(np.float64).reshape(shape)
        off += n
    return out


def _sig(x):
    return 1 / (1 + np.exp(-x))


def _silu(x):
    return x * _sig(x)


def legendre(l, x):
    return [1.0, x, 0.5 * (3 * x * x - 1)][l]


def closed_form_atom_energies(pos, sp, hp, blob, K):
    """Direct evaluation of the K = 1 or K = 2 model for a non-periodic
    cluster, with bond-angle Legendre polynomials in place of harmonics:
    sum_m Y_lm(u) Y_lm(v) = (2l+1) P_l(u.v) and C^(0,l,l) = C^(l,l,0) = I/sqrt(2l+1)."""
    w = _unpack(blob, hp)
    C, L, N = hp.channels, hp.l_max, len(pos)
    inv_n = 1 / hp.avg_neighbors
    nbr = {i: [] for i in range(N)}
    for i in range(N):
        for j in range(N):
            if i != j:
                r = pos[j] - pos[i]
                d = math.sqrt(r @ r)
                if d < RC:
                    nbr[i].append((j, r / d, d))

    def R(t, d, path_idx):
        e, _ = oracle.radial_features(np.array([d]), RC, hp.n_basis, hp.envelope_p)
        a = _silu(_silu(e[0] @ w[f"L{t}.W1"]) @ w[f"L{t}.W2"])
        out = a @ w[f"L{t}.W3"]
        return out[path_idx * C:(path_idx + 1) * C]

    h0 = w["W_emb"][sp]
    ht1 = w["W_emb"] @ w["L1.W_up0"]            # per-species table
    # layer 1: paths (0,l,l) are columns l of W3 (layer 1 input is scalar)
    A10 = np.array([inv_n * sum(R(1, d, 0) * ht1[sp[k]] for k, _, d in nbr[j]) if nbr[j]
                    else np.zeros(C) for j in range(N)])
    z10 = A10 @ w["L1.W_down0"]
    h10 = h0 + _silu(z10[:, :C])
    if K == 1:
        return w["e0"][sp] + h10 @ w["w_read"]

    def T1(j, l, v):
        """sum_m A1[j, :, l m] Y_lm(v)"""
        acc = np.zeros(C)
        for k, ujk, d in nbr[j]:
            acc += R(1, d, l) * ht1[sp[k]] * math.sqrt(2 * l + 1) * legendre(l, ujk @ v)
        return inv_n * acc

    # layer-2 paths (l,l,0): index in the t>=2 path list
    idx2 = {l: [p for p in _paths2(L)].index((l, l, 0)) for l in range(L + 1)}
    ht20 = h10 @ w["L2.W_up0"]
    E = np.zeros(N)
    for i in range(N):
        A2 = np.zeros(C)
        for j, uij, d in nbr[i]:
            msg = R(2, d, idx2[0]) * ht20[j]
            for l in range(1, L + 1):
                gate = _sig(z10[j, l * C:(l + 1) * C])
                proj = ((gate * (T1(j, l, uij) @ w[f"L1.W_down{l}"])) @ w[f"L2.W_up{l}"])
                msg = msg + R(2, d, idx2[l]) * proj / math.sqrt(2 * l + 1)
            A2 += inv_n * msg
        z2 = A2 @ w["L2.W_down0"][:, :C]
        E[i] = w["e0"][sp[i]] + (h10[i] + _silu(z2)) @ w["w_read"]
    return E


def _paths2(L):
    return [(a, b, c) for a in range(L + 1) for b in range(L + 1) for c in range(L + 1)
            if (a + b + c) % 2 == 0 and abs(a - b) <= c <= a + b]


@pytest.mark.parametrize("L,T,K", [(1, 2, 1), (1, 2, 2), (2, 2, 2), (2, 4, 2), (2, 3, 1)])
def test_closed_form_body_order_expansion(L, T, K):
    pos, sp = cluster(14, 10 + L + T)
    hp = hp_of(L, 8, T)
    blob = W.make_weights(hp, 5, e0=[0.3, -0.2, 0.1])
    ref = closed_form_atom_energies(pos, sp, hp, blob, K)
    res = ev(pos, sp, hp, blob, K=K, forces=False)
    assert np.allclose(res.atom_energy, ref, rtol=0, atol=1e-12)
    assert res.energy == pytest.approx(ref.sum(), abs=1e-11)


# ------------------------------------------------------------- derivatives

@pytest.mark.parametrize("L,C,T,K", [(1, 32, 2, 2), (2, 16, 3, 3)])
def test_forces_match_finite_differences(L, C, T, K):
    s = W.small_system()
    hp = hp_of(L, C, T, S=2)
    blob = W.make_weights(hp, 103)
    res = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp, K=K)
    h = 1e-5
    rng = np.random.default_rng(0)
    for a in rng.choice(128, 4, replace=False):
        for k in range(3):
            p = s.positions.copy()
            p[a, k] += h
            ep = oracle.evaluate(p, s.species, s.cell, s.pbc, blob, hp, K=K, forces=False).energy
            p[a, k] -= 2 * h
            em = oracle.evaluate(p, s.species, s.cell, s.pbc, blob, hp, K=K, forces=False).energy
            assert -(ep - em) / (2 * h) == pytest.approx(res.forces[a, k], abs=2e-9)
    assert np.allclose(res.forces.sum(axis=0), 0.0, atol=1e-12)


def test_virial_matches_strain_finite_differences():
    s = W.small_system()
    hp = W.HP_SMALL
    blob = W.make_weights(hp, 103)
    res = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp)
    assert np.allclose(res.virial, res.virial.T, atol=1e-12)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            vals = []
            for sgn in (1, -1):
                eps = np.zeros((3, 3))
                eps[a, b] = sgn * h
                M = np.eye(3) + eps
                vals.append(oracle.evaluate(s.positions @ M.T, s.species, s.cell @ M.T, s.pbc,
                                            blob, hp, forces=False).energy)
            dEde = (vals[0] - vals[1]) / (2 * h)
            assert -dEde == pytest.approx(res.virial[a, b], abs=1e-8)


# ------------------------------------------------------------- symmetries

def test_rotation_translation_permutation():
    s = W.small_system()
    hp = W.HP_SMALL
    blob = W.make_weights(hp, 103)
    base = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp)
    scale = np.abs(base.forces).max()
    rng = np.random.default_rng(7)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = q @ np.diag(np.sign(np.diag(r)))
    rot = oracle.evaluate(s.positions @ Q.T, s.species, s.cell @ Q.T, s.pbc, blob, hp)
    assert rot.energy == pytest.approx(base.energy, rel=1e-12)
    assert np.allclose(rot.forces, base.forces @ Q.T, atol=1e-12 * max(1, scale))
    assert np.allclose(rot.virial, Q @ base.virial @ Q.T, atol=1e-11)
    tr = oracle.evaluate(s.positions + np.array([3.3, -7.1, 100.2]), s.species, s.cell, s.pbc, blob, hp)
    assert tr.energy == pytest.approx(base.energy, rel=1e-12)
    assert np.allclose(tr.forces, base.forces, atol=1e-12)
    perm = rng.permutation(128)
    pe = oracle.evaluate(s.positions[perm], s.species[perm], s.cell, s.pbc, blob, hp)
    assert pe.energy == pytest.approx(base.energy, rel=1e-12)
    assert np.allclose(pe.forces, base.forces[perm], atol=1e-12)
    assert np.allclose(pe.atom_energy, base.atom_energy[perm], atol=1e-12)
    # improper rotation (inversion): natural-parity paths make E O(3)-invariant
    inv = oracle.evaluate(-s.positions, s.species, -s.cell, s.pbc, blob, hp)
    assert inv.energy == pytest.approx(base.energy, rel=1e-12)
    assert np.allclose(inv.forces, -base.forces, atol=1e-12)


def test_dimer():
    hp = hp_of(2, 16, 2)
    blob = W.make_weights(hp, 9)
    sp = np.array([0, 2], np.int32)
    rng = np.random.default_rng(1)
    E = []
    for d in (2.2, 2.2, 3.7):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0]]) + np.array([[0, 0, 0], d * u])
        res = ev(pos, sp, hp, blob)
        assert np.allclose(res.forces[0], -res.forces[1], atol=1e-14)
        assert np.linalg.norm(np.cross(res.forces[0], u)) < 1e-12 * max(1, np.linalg.norm(res.forces[0]))
        E.append(res.energy)
    assert E[0] == pytest.approx(E[1], rel=1e-13)
    assert E[0] != pytest.approx(E[2], rel=1e-6)


def test_separability():
    hp = hp_of(2, 8, 3)
    blob = W.make_weights(hp, 11)
    p1, s1 = cluster(10, 1)
    p2, s2 = cluster(9, 2)
    p2 = p2 + np.array([40.0, 0, 0])       # farther apart than K*r_cut = 15
    a = ev(p1, s1, hp, blob).energy
    b = ev(p2, s2, hp, blob).energy
    both = ev(np.vstack([p1, p2]), np.concatenate([s1, s2]), hp, blob)
    assert both.energy == pytest.approx(a + b, rel=1e-13)


def test_depth_pruning_is_truncation():
    """K < T reads out from layer K with the unchanged weights of layers
    1..K (Methods, "Message Passing Depth Pruning")."""
    pos, sp = cluster(16, 3)
    hp6, hp2 = hp_of(2, 8, 6), hp_of(2, 8, 2)
    blob6 = W.make_weights(hp6, 12)
    lay6 = W.weight_layout(hp6)
    sizes = [int(np.prod(s)) for _, s, _ in lay6]
    offs = np.cumsum([0] + sizes)
    keep = [k for k, (name, _, _) in enumerate(lay6)
            if not name.startswith(("L3.", "L4.", "L5.", "L6."))]
    blob2 = np.concatenate([blob6[offs[k]:offs[k + 1]] for k in keep])
    assert blob2.size == W.weights_count(hp2)
    a = ev(pos, sp, hp6, blob6, K=2)
    b = ev(pos, sp, hp2, blob2, K=2)
    assert a.energy == b.energy
    assert np.array_equal(a.forces, b.forces)
    c = ev(pos, sp, hp6, blob6, K=6)
    assert c.energy != pytest.approx(a.energy, rel=1e-6)


# ------------------------------------------------------------- partitions

def _slab_case():
    s = W.slab_full_system(40, 6, 6, 31, 32)       # 1440 atoms, 13.6 x 13.6 A cross-section
    hp = hp_of(2, 8, 2)
    return s, hp, W.make_weights(hp, 33)


def test_partition_root_energies_and_force_sum():
    """8 slab partitions with a K*r_cut halo: (i) root-atom energies equal the
    full system's; (ii) energies, forces (ghost rows returned to owners) and
    virials summed over partitions equal the full-system values."""
    s, hp, blob = _slab_case()
    full = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp)
    E, F, Wv, parts = oracle.evaluate_partitioned(s.positions, s.species, s.cell, blob, hp,
                                                  K=2, n_parts=8, halo=2 * RC)
    for res, gi, n_own in parts:
        assert np.allclose(res.atom_energy[:n_own], full.atom_energy[gi[:n_own]], atol=1e-12)
    owned = np.concatenate([gi[:n] for _, gi, n in parts])
    assert np.array_equal(np.sort(owned), np.arange(s.n_atoms))
    assert E == pytest.approx(full.energy, abs=1e-9)
    assert np.allclose(F, full.forces, atol=1e-12)
    assert np.allclose(Wv, full.virial, atol=1e-10)


def _reach(s, roots, K):
    """Atoms within K hops of the roots from powers of the adjacency matrix
    of a brute-force minimum-image distance matrix (no neighbour list, no
    breadth-first levels)."""
    L = np.diag(s.cell)
    d = s.positions[:, None, :] - s.positions[None, :, :]
    d -= np.round(d / L) * L
    A = (np.sqrt((d ** 2).sum(-1)) < RC).astype(np.int64)
    np.fill_diagonal(A, 0)
    r = np.zeros(s.n_atoms, dtype=np.int64)
    r[roots] = 1
    for _ in range(K):
        r = ((r + A @ r) > 0).astype(np.int64)
    return r.astype(bool)


@pytest.mark.parametrize("K", [1, 2])
def test_bfs_share_is_the_k_hop_set(K):
    """The graph halo (stage-2 breadth-first expansion): the halo atoms are
    exactly the atoms within K hops of a root, each once, in the rows of the
    geometric K*r_cut share (same positions, same order)."""
    s, _, _ = _slab_case()
    for part in (0, 5):
        lp, ls, pbc, n_own, gi = oracle.bfs_share(s.positions, s.species, s.cell, 8, part, K, RC)
        gp, gs, _, g_own, ggi = oracle.slab_share(s.positions, s.species, s.cell, 8, part, K * RC)
        assert n_own == g_own and np.array_equal(gi[:n_own], ggi[:n_own])
        want = _reach(s, gi[:n_own], K)
        want[gi[:n_own]] = False
        assert np.array_equal(np.sort(gi[n_own:]), np.flatnonzero(want))
        keep = np.isin(np.arange(gp.shape[0]), np.arange(g_own)) | want[ggi]
        assert np.array_equal(lp, gp[keep]) and np.array_equal(gi, ggi[keep]) and np.array_equal(ls, gs[keep])
        assert not pbc[0] and pbc[1] and pbc[2]


def test_bfs_share_partition_rule():
    """Graph-halo partitions reproduce the full system: root-atom energies,
    and forces / virials summed over partitions with ghost rows returned to
    their owners; the graph halo is smaller than the geometric one."""
    s, hp, blob = _slab_case()
    full = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp)
    F = np.zeros_like(full.forces)
    E, Wv, rows_bfs, rows_geo = 0.0, np.zeros((3, 3)), 0, 0
    for part in range(8):
        lp, ls, pbc, n_own, gi = oracle.bfs_share(s.positions, s.species, s.cell, 8, part, 2, RC)
        rows_bfs += lp.shape[0]
        rows_geo += oracle.slab_share(s.positions, s.species, s.cell, 8, part, 2 * RC)[0].shape[0]
        r = oracle.evaluate(lp, ls, s.cell, pbc, blob, hp, K=2, n_owned=n_own)
        assert np.allclose(r.atom_energy[:n_own], full.atom_energy[gi[:n_own]], atol=1e-12)
        np.add.at(F, gi, r.forces)
        E += r.energy
        Wv += r.virial
    assert E == pytest.approx(full.energy, abs=1e-9)
    assert np.allclose(F, full.forces, atol=1e-12)
    assert np.allclose(Wv, full.virial, atol=1e-10)
    assert rows_bfs < rows_geo


def test_bfs_share_rejects_wrapped_halo():
    s, _, _ = _slab_case()
    with pytest.raises(ValueError):
        oracle.bfs_share(s.positions, s.species, s.cell, 2, 0, 6, RC)


def test_partition_alone_needs_double_halo():
    """(iii) one partition on its own reproduces its root atoms' forces only
    if its halo is 2*K*r_cut deep and the energy is summed over the root
    atoms plus the ghosts within K*r_cut of the slab (the root atoms' forces
    also carry the gradient of those neighbours' energies).  Summing only
    root energies, the atoms near the faces miss that gradient."""
    s, hp, blob = _slab_case()
    full = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp)
    Lx = s.cell[0, 0]
    lo, hi = 3 * Lx / 8, 4 * Lx / 8
    lp, ls, pbc, n_own, gi = oracle.slab_share(s.positions, s.species, s.cell, 8, 3, 4 * RC)
    dist = np.maximum(np.maximum(lo - lp[:, 0], lp[:, 0] - hi), 0.0)
    ghosts = np.arange(n_own, lp.shape[0])
    inner = ghosts[dist[ghosts] < 2 * RC]
    outer = ghosts[dist[ghosts] >= 2 * RC]
    order = np.concatenate([np.arange(n_own), inner, outer])
    lp, ls, gi = lp[order], ls[order], gi[order]
    ref = full.forces[gi[:n_own]]
    wide = oracle.evaluate(lp, ls, s.cell, pbc, blob, hp, K=2, n_owned=n_own + inner.size)
    assert np.abs(wide.forces[:n_own] - ref).max() < 1e-12
    roots_only = oracle.evaluate(lp, ls, s.cell, pbc, blob, hp, K=2, n_owned=n_own)
    assert np.abs(roots_only.forces[:n_own] - ref).max() > 1e-6


def test_local_cluster_force():
    s = W.bulk_system(18, 5, 6)                     # 40.9 A box: 2*K*r_cut = 20 A fits
    hp = hp_of(2, 8, 2)
    blob = W.make_weights(hp, 7)
    full = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp)
    for a in (0, 2917):
        lp, ls, n_own, gi, c = oracle.local_cluster(s.positions, s.species, s.cell, a, 4 * RC, 2 * RC)
        res = oracle.evaluate(lp, ls, np.eye(3), [False] * 3, blob, hp, K=2, n_owned=n_own)
        assert np.allclose(res.forces[c], full.forces[a], atol=1e-12)
        assert res.atom_energy[c] == pytest.approx(full.atom_energy[a], abs=1e-12)


# ------------------------------------------------- every middle-layer path (K = 3, l_max = 2)

def _scipy_real_harmonics(l, v):
    """A real orthonormal basis of the degree-l harmonics built from scipy's
    complex ones (its own phase convention): sqrt(2) Re Y_l^m for m > 0,
    Y_l^0, sqrt(2) Im Y_l^|m| for m < 0, scaled by sqrt(4 pi) to the
    component normalisation.  It differs from the oracle's basis by an
    orthogonal matrix per degree, which leaves every energy unchanged when the
    coupling tensors are built from the same basis."""
    from scipy.special import sph_harm_y
    x, y, z = v
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    out = []
    for m in range(-l, l + 1):
        c = complex(sph_harm_y(l, abs(m), theta, phi))
        out.append(c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag))
    return math.sqrt(4 * math.pi) * np.array(out)


def _scipy_couplings(L):
    """C = G / ||G||_F of the Gaunt integrals in the scipy basis, by a product
    rule (12 Gauss-Legendre nodes in cos(theta) x 24 in phi: exact to degree
    23, the integrands have degree <= 6)."""
    zs, wz = np.polynomial.legendre.leggauss(12)
    pts, wts = [], []
    for z, wzz in zip(zs, wz):
        for k in range(24):
            ph = 2 * math.pi * k / 24
            s = math.sqrt(1 - z * z)
            pts.append((s * math.cos(ph), s * math.sin(ph), z))
            wts.append(wzz * 2 * math.pi / 24)
    Ys = [{l: _scipy_real_harmonics(l, p) for l in range(L + 1)} for p in pts]
    out = {}
    for a, b, c in _paths2(L):
        G = sum(wq * np.einsum("x,y,z->xyz", Yq[a], Yq[b], Yq[c]) for wq, Yq in zip(wts, Ys))
        out[(a, b, c)] = G / np.linalg.norm(G)
    return out


def independent_atom_energies(pos, sp, hp, blob, K):
    """The layer equations written out edge by edge for a non-periodic
    cluster: every path at every layer (dead ones included), every gate, the
    radial basis and envelope retyped from their definitions, the harmonics and
    couplings from scipy in its own basis; shares only the blob layout."""
    w = _unpack(blob, hp)
    C, L = hp.channels, hp.l_max
    rc, nb, inv_n, N = hp.r_cut, hp.n_basis, 1.0 / hp.avg_neighbors, len(pos)
    cpl = _scipy_couplings(L)

    def radial(t, d):
        x = d / rc
        env = 1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8
        e = np.array([env * math.sqrt(2 / rc) * math.sin(n * math.pi * d / rc) / d for n in range(1, nb + 1)])
        return _silu(_silu(e @ w[f"L{t}.W1"]) @ w[f"L{t}.W2"]) @ w[f"L{t}.W3"]

    nbr = []
    for i in range(N):
        row = []
        for j in range(N):
            r = pos[j] - pos[i]
            d = math.sqrt(r @ r)
            if i != j and d < rc:
                row.append((j, r / d, d))
        nbr.append(row)
    h = {l: np.zeros((N, 2 * l + 1, C)) for l in range(L + 1)}
    h[0][:, 0, :] = w["W_emb"][sp]
    for t in range(1, K + 1):
        l_in = [0] if t == 1 else list(range(L + 1))
        paths = [p for p in _paths2(L) if p[0] in l_in]
        ht = {l: h[l] @ w[f"L{t}.W_up{l}"] for l in l_in}
        A = {l: np.zeros((N, 2 * l + 1, C)) for l in range(L + 1)}
        for i in range(N):
            for j, u, d in nbr[i]:
                R = radial(t, d).reshape(len(paths), C)
                Y = {l: _scipy_real_harmonics(l, u) for l in range(L + 1)}
                for q, (a, b, c) in enumerate(paths):
                    A[c][i] += inv_n * R[q] * np.einsum("xyz,xk,y->zk", cpl[(a, b, c)], ht[a][j], Y[b])
        z0 = A[0][:, 0, :] @ w[f"L{t}.W_down0"]
        hn = {0: h[0] + _silu(z0[:, :C])[:, None, :]}
        for l in range(1, L + 1):
            gate = _sig(z0[:, l * C:(l + 1) * C])
            hn[l] = h[l] + gate[:, None, :] * (A[l] @ w[f"L{t}.W_down{l}"])
        h = hn
    return w["e0"][sp] + h[0][:, 0, :] @ w["w_read"]


def test_independent_deep_forward_every_path():
    """K = 3, l_max = 2: the middle layer runs all 11 coupling paths, and its
    per-atom energies equal the independent edge-by-edge evaluation."""
    pos, sp = cluster(9, 41, box=6.0, dmin=1.5)
    hp = hp_of(2, 4, 3)
    blob = W.make_weights(hp, 17, e0=[0.2, -0.1, 0.05])
    ref = independent_atom_energies(pos, sp, hp, blob, 3)
    res = ev(pos, sp, hp, blob, K=3, forces=False)
    assert np.allclose(res.atom_energy, ref, rtol=0, atol=1e-12)
    # every middle-layer path contributes: dropping any one moves the energy
    base = res.energy
    for p in _paths2(2):
        if p == (0, 0, 0):
            continue
        with _planted_coupling(p, lambda Cp: 0.0 * Cp):
            dropped = ev(pos, sp, hp, blob, K=3, forces=False).energy
        assert abs(dropped - base) > 1e-10, p


class _planted_coupling:
    """Replace the oracle's coupling tensor of one path inside a with-block
    (a deliberate mistake, to show that a pin notices it)."""

    def __init__(self, path, fn):
        self.path, self.fn = path, fn

    def __enter__(self):
        import oracle.model as om
        self.om, self.orig = om, om.coupling_tensor

        def patched(a, b, c):
            Cp = self.orig(a, b, c)
            return self.fn(np.array(Cp)) if (a, b, c) == self.path else Cp
        om.coupling_tensor = patched
        return self

    def __exit__(self, *exc):
        self.om.coupling_tensor = self.orig
        return False


def _o3_deviation(pos, sp, cell, pbc, hp, blob, K):
    """Largest relative deviation of E, E_i, F and W from their required
    behaviour under a proper rotation, the inversion, a translation and a
    permutation."""
    base = oracle.evaluate(pos, sp, cell, pbc, blob, hp, K=K)
    fs = max(np.abs(base.forces).max(), 1e-30)
    es = max(np.abs(base.atom_energy).max(), 1e-30)
    ws = max(np.abs(base.virial).max(), 1e-30)
    rng = np.random.default_rng(3)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    dev = 0.0
    for M in (Q, -np.eye(3), -Q):
        o = oracle.evaluate(pos @ M.T, sp, cell @ M.T, pbc, blob, hp, K=K)
        dev = max(dev, np.abs(o.atom_energy - base.atom_energy).max() / es,
                  np.abs(o.forces - base.forces @ M.T).max() / fs,
                  np.abs(o.virial - M @ base.virial @ M.T).max() / ws)
    tr = oracle.evaluate(pos + np.array([1.7, -2.9, 40.3]), sp, cell, pbc, blob, hp, K=K)
    dev = max(dev, np.abs(tr.atom_energy - base.atom_energy).max() / es,
              np.abs(tr.forces - base.forces).max() / fs)
    perm = rng.permutation(len(pos))
    pe = oracle.evaluate(pos[perm], sp[perm], cell, pbc, blob, hp, K=K)
    dev = max(dev, np.abs(pe.atom_energy - base.atom_energy[perm]).max() / es,
              np.abs(pe.forces - base.forces[perm]).max() / fs)
    return dev


@pytest.mark.parametrize("periodic", [False, True])
def test_rotation_inversion_translation_deep(periodic):
    """O(3) invariance of E and E_i, equivariance of F and W, at T = K = 3,
    l_max = 2, so the paths (1,0,1) (1,1,2) (1,2,1) (2,0,2) (2,1,1) (2,2,2)
    of the middle layer carry features of degree 1 and 2 into it."""
    hp = hp_of(2, 8, 3)
    blob = W.make_weights(hp, 23)
    if periodic:
        rng = np.random.default_rng(12)
        box = 10.5
        pos = W.lattice_positions(4, 4, 4, box / 4, 31)
        sp = rng.integers(0, 3, 64).astype(np.int32)
        cell, pbc = np.eye(3) * box, (True, True, True)
    else:
        pos, sp = cluster(20, 77, box=8.0, dmin=1.5)
        cell, pbc = np.eye(3) * 100.0, (False, False, False)
    assert _o3_deviation(pos, sp, cell, np.array(pbc), hp, blob, 3) < 1e-11


@pytest.mark.parametrize("path", [(1, 1, 2), (1, 2, 1), (2, 1, 1), (2, 2, 2)])
def test_deep_pins_notice_a_planted_mistake(path):
    """A wrong m order in one middle-layer coupling (a cyclic shift of its
    first index, as a mis-ordered harmonic block would give) breaks both the
    O(3) pin and the independent forward."""
    pos, sp = cluster(9, 41, box=6.0, dmin=1.5)
    hp = hp_of(2, 4, 3)
    blob = W.make_weights(hp, 17)
    ref = independent_atom_energies(pos, sp, hp, blob, 3)
    with _planted_coupling(path, lambda Cp: np.roll(Cp, 1, axis=0)):
        bad = ev(pos, sp, hp, blob, K=3, forces=False)
        dev = _o3_deviation(pos, sp, np.eye(3) * 100.0, np.array([False] * 3), hp, blob, 3)
    # the clean oracle agrees to 1e-12 (energies) and 1e-11 (O(3) deviation);
    # the planted mistake moves them by 3e-10 .. 6e-10 and 1.7e-7 .. 6.5e-7
    assert np.abs(bad.atom_energy - ref).max() > 1e-10
    assert dev > 1e-8
