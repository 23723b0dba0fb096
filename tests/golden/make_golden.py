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


JOBS = {"mpdp_K2": lambda: mpdp(2), "mpdp_K6": lambda: mpdp(6),
        "slab20k_K2": lambda: slab_downscale(2), "slab20k_K6": lambda: slab_downscale(6)}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
