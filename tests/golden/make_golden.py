"""Write the stored oracle outputs used by the GPU parity tests.

Every value here comes from ``oracle/`` (FP64) on the seeded workloads of
``workloads/``; nothing is taken from the GPU path.  Run from the repository
root:  python tests/golden/make_golden.py [name ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle            # noqa: E402
import workloads as W    # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def save(name, res, extra=None):
    d = {"energy": np.float64(res.energy), "forces": res.forces, "virial": res.virial,
         "atom_energy": res.atom_energy, "n_edges": np.int64(res.n_edges)}
    if extra:
        d.update(extra)
    tmp = os.path.join(OUT, name + ".tmp.npz")
    np.savez_compressed(tmp, **d)
    os.replace(tmp, os.path.join(OUT, name + ".npz"))


def mpdp(K):
    s = W.mpdp_system()
    blob = W.make_weights(W.HP_MPDP, W.WEIGHT_SEEDS["mpdp"])
    t = time.time()
    res = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, W.HP_MPDP, K=K)
    print(f"mpdp K={K}: {time.time() - t:.1f}s E={res.energy:.10f} edges={res.n_edges}")
    save(f"mpdp_K{K}", res, {"seconds": np.float64(time.time() - t)})


def slab_downscale(K):
    s = W.slab_downscale_full()
    hp = W.HP_MPDP
    blob = W.make_weights(hp, W.WEIGHT_SEEDS["slab8m"])
    t = time.time()
    res = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, hp, K=K)
    print(f"slab20k K={K}: {time.time() - t:.1f}s E={res.energy:.10f} edges={res.n_edges}")
    save(f"slab20k_K{K}", res)


def bulk32k():
    """32^3 = 32,768 atoms of the 1M-atom box's lattice, density and species
    mix, with its potential (C = 128, l_max = 2, K = 2): every atom of a
    periodic box evaluated by the oracle."""
    s = W.bulk_system(32, 311, 312)
    blob = W.make_weights(W.HP_BULK, W.WEIGHT_SEEDS["bulk1m"])
    t = time.time()
    res = oracle.evaluate(s.positions, s.species, s.cell, s.pbc, blob, W.HP_BULK, K=2)
    print(f"bulk32k K=2: {time.time() - t:.1f}s E={res.energy:.10f} edges={res.n_edges}")
    save("bulk32k_K2", res, {"seconds": np.float64(time.time() - t)})


# centers of the local clusters cut from the 1M-atom box: eight atoms spread
# over the box (and so over the spatially sorted row order of the GPU path)
BULK1M_CENTERS = (1234, 130017, 262626, 387421, 505050, 631579, 777777, 912345)
BULK1M_RADIUS = 24.0


def bulk1m_clusters():
    """Exact full-system values of the 1M-atom box at K = 2 from non-periodic
    clusters of radius 24 A around eight atoms: with the energy summed over
    the atoms within radius - K r_c, the energies of those atoms are exact and
    the forces of the atoms within radius - 2 K r_c are exact (each message
    hop is shorter than r_c)."""
    s = W.bulk1m_system()
    hp, K = W.HP_BULK, 2
    blob = W.make_weights(hp, W.WEIGHT_SEEDS["bulk1m"])
    rc, R = hp.r_cut, BULK1M_RADIUS
    f_idx, f_val, e_idx, e_val, cen = [], [], [], [], []
    t = time.time()
    for a in BULK1M_CENTERS:
        lp, ls, n_in, gi, c = oracle.local_cluster(s.positions, s.species, s.cell, a, R, R - K * rc)
        r = oracle.evaluate(lp, ls, np.eye(3), [False] * 3, blob, hp, K=K, n_owned=n_in)
        dist = np.linalg.norm(lp - lp[c], axis=1)
        exact = np.flatnonzero(dist <= R - 2 * K * rc)
        f_idx.append(gi[exact]); f_val.append(r.forces[exact])
        e_idx.append(gi[:n_in]); e_val.append(r.atom_energy[:n_in])
        cen.append(np.full(exact.size, a))
        print(f"center {a}: {lp.shape[0]} atoms, {exact.size} exact forces, {n_in} exact energies, "
              f"{time.time() - t:.1f}s")
    tmp = os.path.join(OUT, "bulk1m_clusters.tmp.npz")
    np.savez_compressed(tmp, force_index=np.concatenate(f_idx), forces=np.concatenate(f_val),
                        force_center=np.concatenate(cen), energy_index=np.concatenate(e_idx),
                        atom_energy=np.concatenate(e_val), centers=np.array(BULK1M_CENTERS),
                        radius=np.float64(R))
    os.replace(tmp, os.path.join(OUT, "bulk1m_clusters.npz"))


JOBS = {"mpdp_K2": lambda: mpdp(2), "mpdp_K6": lambda: mpdp(6),
        "slab20k_K2": lambda: slab_downscale(2), "slab20k_K6": lambda: slab_downscale(6),
        "bulk32k_K2": bulk32k, "bulk1m_clusters": bulk1m_clusters}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
