"""Energy, forces and virial of the equivariant message-passing potential
(oracle, float64, analytic backward).

Notation: atoms i (receiver) and j (sender) of edge e = (i, j, S);
r_e = x_j - x_i + S.cell, d_e = |r_e|, u_e = r_e / d_e; features h[i, lm, c]
with flat harmonic index lm = l^2 + (m + l) and channel c.

Forward, layer t = 1..K (the first K of the T layers in the weight set;
message-passing depth pruning keeps the first K layers and reads out from
layer K):
  1. ht[j, l] = h[j, l] @ W_up[t, l]                   (channel mixing per l)
  2. R_e = silu(silu(e_e @ W1) @ W2) @ W3             ([P, C] per edge, no bias)
  3. A[i, l3 m3, c] = (1/n_avg) sum_{e: recv(e)=i} sum_{p=(l1,l2,l3)}
          R_e[p, c] sum_{m1, m2} C^p[m1, m2, m3] ht[j, l1 m1, c] Y^l2_m2(u_e)
  4. z0 = A[:, 0] @ W_down[t, 0]  (C features, then one gate block per l>=1);
     z_l = A[:, l] @ W_down[t, l]   (per m)
  5. h'[:, 0] = h[:, 0] + silu(z0[:, :C]);
     h'[:, l] = h[:, l] + sigmoid(z0[:, lC:(l+1)C]) * z_l    (l >= 1)
  At layer K only l3 = 0 outputs are needed (only scalars are read out).
Readout: E_i = e0[z_i] + h^(K)[i, 0] . w_read;  E = sum over owned atoms
(the first n_owned; Methods "Global Output Integration": the energy of a
partition is the sum of its root-node energies).

Backward (reverse order, written out by hand):
  dE/dh^(K)[i,0] = w_read for owned atoms, 0 for ghost atoms; residual
  connections pass the adjoint through; gates and linear maps transpose;
  per edge the adjoints of R, of ht[j] and of Y(u_e) follow from step 3;
  the radial MLP is differentiated back to e_e; then
    g_e = dE/dr_e = (dE/dd_e) u_e + (I - u u^T)/d_e (dP/du)^T dE/dY
  Forces F_i = sum_{recv(e)=i} g_e - sum_{send(e)=i} g_e;
  virial W = -sum_e r_e (x) g_e.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .gaunt import coupling_tensor, layer_paths, live_paths
from .neighbors import edge_vectors, neighbor_list
from .radial import radial_features
from .sh import real_sh, real_sh_grad
from .weights import parse_weights


@dataclasses.dataclass
class Result:
    energy: float
    forces: np.ndarray        # [N, 3]
    virial: np.ndarray        # [3, 3]
    atom_energy: np.ndarray   # [N]
    n_edges: int


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def silu(x):
    return x * sigmoid(x)


def dsilu(x):
    s = sigmoid(x)
    return s * (1.0 + x * (1.0 - s))


def blk(l: int) -> slice:
    return slice(l * l, (l + 1) * (l + 1))


def segment_sum(index: np.ndarray, values: np.ndarray, n: int) -> np.ndarray:
    """out[k] = sum of values[e] over e with index[e] == k (stable order)."""
    out = np.zeros((n,) + values.shape[1:])
    if index.size == 0:
        return out
    order = np.argsort(index, kind="stable")
    idx = index[order]
    starts = np.flatnonzero(np.r_[True, idx[1:] != idx[:-1]])
    out[idx[starts]] = np.add.reduceat(values[order], starts, axis=0)
    return out


def _yc(Cp: np.ndarray, Yb: np.ndarray) -> np.ndarray:
    """YC[e, m1, m3] = sum_m2 C[m1, m2, m3] Y[e, m2]."""
    return np.einsum("abk,eb->eak", Cp, Yb)


def evaluate(positions, species, cell, pbc, blob, hp, K: Optional[int] = None,
             n_owned: Optional[int] = None, edges=None, chunk: int = 8192,
             forces: bool = True) -> Result:
    positions = np.asarray(positions, dtype=np.float64)
    species = np.asarray(species, dtype=np.int64)
    N = positions.shape[0]
    K = hp.n_layers if K is None else int(K)
    if not 1 <= K <= hp.n_layers:
        raise ValueError("K must be in 1..n_layers")
    n_owned = N if n_owned is None else int(n_owned)
    w = parse_weights(blob, hp)
    C, L, H = hp.channels, hp.l_max, hp.radial_hidden
    nlm = (L + 1) ** 2
    inv_n = 1.0 / hp.avg_neighbors

    if edges is None:
        ei, ej, eS = neighbor_list(positions, cell, pbc, hp.r_cut)
    else:
        ei, ej, eS = (np.asarray(a) for a in edges)
        order = np.lexsort((eS[:, 2], eS[:, 1], eS[:, 0], ej, ei))
        ei, ej, eS = ei[order], ej[order], eS[order]
    E = ei.size
    r = edge_vectors(positions, cell, ei, ej, eS)
    d = np.sqrt(np.sum(r * r, axis=1))
    if np.any(d == 0.0):
        raise ValueError("coincident atoms")
    u = r / d[:, None]
    Y = real_sh(u, L)
    ef, def_ = radial_features(d, hp.r_cut, hp.n_basis, hp.envelope_p)
    chunks = [slice(a, min(E, a + chunk)) for a in range(0, E, chunk)]

    def mlp(lay, live, sl):
        p1 = ef[sl] @ lay["W1"]
        a1 = silu(p1)
        p2 = a1 @ lay["W2"]
        a2 = silu(p2)
        W3 = lay["W3"][:, [k for k, _ in live], :]            # [H, P_live, C]
        R = (a2 @ W3.reshape(W3.shape[0], -1)).reshape(a2.shape[0], W3.shape[1], W3.shape[2])
        return p1, a1, p2, a2, W3, R

    # ---------------- forward ----------------
    h = np.zeros((N, nlm, C))
    h[:, 0, :] = w["W_emb"][species]
    cache = []
    for t in range(1, K + 1):
        lay = w["layers"][t - 1]
        l_in = [0] if t == 1 else list(range(L + 1))
        live = live_paths(t, K, L)
        ht = np.zeros((N, nlm, C))
        for l in l_in:
            ht[:, blk(l), :] = h[:, blk(l), :] @ lay["W_up"][l]
        A = np.zeros((N, nlm, C))
        for sl in chunks:
            R = mlp(lay, live, sl)[-1]
            msg = np.zeros((sl.stop - sl.start, nlm, C))
            for q, (_, (l1, l2, l3)) in enumerate(live):
                yc = _yc(coupling_tensor(l1, l2, l3), Y[sl, blk(l2)])      # [e, m1, m3]
                hj = ht[ej[sl]][:, blk(l1), :]                              # [e, m1, c]
                msg[:, blk(l3), :] += np.matmul(yc.transpose(0, 2, 1), hj) * R[:, q, None, :]
            A += segment_sum(ei[sl], msg, N)
        A *= inv_n
        z0 = A[:, 0, :] @ lay["W_down"][0]
        zl = {}
        hn = h.copy()
        hn[:, 0, :] = h[:, 0, :] + silu(z0[:, :C])
        if t < K:
            for l in range(1, L + 1):
                zl[l] = A[:, blk(l), :] @ lay["W_down"][l]
                gate = sigmoid(z0[:, l * C:(l + 1) * C])
                hn[:, blk(l), :] = h[:, blk(l), :] + gate[:, None, :] * zl[l]
        cache.append({"ht": ht, "z0": z0, "zl": zl, "live": live, "l_in": l_in})
        h = hn
    atom_energy = w["e0"][species] + h[:, 0, :] @ w["w_read"]
    energy = float(np.sum(atom_energy[:n_owned]))
    if not forces:
        return Result(energy, np.zeros((N, 3)), np.zeros((3, 3)), atom_energy, E)

    # ---------------- backward ----------------
    hbar = np.zeros((N, nlm, C))
    hbar[:n_owned, 0, :] = w["w_read"]
    g = np.zeros((E, 3))
    dP = real_sh_grad(u, L)
    for t in range(K, 0, -1):
        lay = w["layers"][t - 1]
        cc = cache[t - 1]
        ht, z0, zl, live, l_in = cc["ht"], cc["z0"], cc["zl"], cc["live"], cc["l_in"]
        zbar0 = np.zeros_like(z0)
        zbar0[:, :C] = hbar[:, 0, :] * dsilu(z0[:, :C])
        Abar = np.zeros((N, nlm, C))
        if t < K:
            for l in range(1, L + 1):
                s = sigmoid(z0[:, l * C:(l + 1) * C])
                Abar[:, blk(l), :] = (hbar[:, blk(l), :] * s[:, None, :]) @ lay["W_down"][l].T
                zbar0[:, l * C:(l + 1) * C] = np.sum(hbar[:, blk(l), :] * zl[l], axis=1) * s * (1.0 - s)
        Abar[:, 0, :] = zbar0 @ lay["W_down"][0].T
        Abar *= inv_n
        htbar = np.zeros((N, nlm, C))
        for sl in chunks:
            p1, a1, p2, a2, W3, R = mlp(lay, live, sl)
            ne = sl.stop - sl.start
            Rbar = np.zeros_like(R)
            Ybar = np.zeros((ne, nlm))
            hjbar = np.zeros((ne, nlm, C))
            Ai = Abar[ei[sl]]
            for q, (_, (l1, l2, l3)) in enumerate(live):
                Cp = coupling_tensor(l1, l2, l3)
                hj = ht[ej[sl]][:, blk(l1), :]
                Ab = Ai[:, blk(l3), :]
                yc = _yc(Cp, Y[sl, blk(l2)])                              # [e, m1, m3]
                T = np.matmul(yc, Ab)                                      # [e, m1, c]
                Rbar[:, q, :] = np.sum(T * hj, axis=1)
                hjbar[:, blk(l1), :] += R[:, q, None, :] * T
                # P[e, m1, m3] = sum_c R[e, c] ht_j[e, m1, c] dA_i[e, m3, c]
                P = np.matmul(hj * R[:, q, None, :], Ab.transpose(0, 2, 1))
                Ybar[:, blk(l2)] += np.einsum("abk,eak->eb", Cp, P)
            htbar += segment_sum(ej[sl], hjbar, N)
            a2bar = Rbar.reshape(ne, -1) @ W3.reshape(W3.shape[0], -1).T
            p2bar = a2bar * dsilu(p2)
            a1bar = p2bar @ lay["W2"].T
            p1bar = a1bar * dsilu(p1)
            ebar = p1bar @ lay["W1"].T
            dbar = np.sum(ebar * def_[sl], axis=1)
            gu = np.einsum("eb,ebk->ek", Ybar, dP[sl])
            ue = u[sl]
            gperp = (gu - ue * np.sum(gu * ue, axis=1, keepdims=True)) / d[sl, None]
            g[sl] += dbar[:, None] * ue + gperp
        hbar_prev = hbar.copy()
        if t >= 2:
            for l in l_in:
                hbar_prev[:, blk(l), :] += htbar[:, blk(l), :] @ lay["W_up"][l].T
        hbar = hbar_prev
    F = segment_sum(ei, g, N) - segment_sum(ej, g, N)
    W = -np.einsum("ea,eb->ab", r, g)
    return Result(energy, F, W, atom_energy, E)
