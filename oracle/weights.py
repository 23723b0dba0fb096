"""Weight-blob parser (oracle's own reading of the packed float32 layout).

Order: W_emb [S, C]; for each layer t = 1..T: W_up[l] [C, C] for each input
degree l ({0} at t = 1, else 0..l_max), W1 [n_b, H], W2 [H, H],
W3 [H, P_t*C] (path-major columns), W_down[0] [C, C*(1+l_max)],
W_down[l] [C, C] for l = 1..l_max; then w_read [C] and e0 [S].
Matrices map rows (inputs) to columns (outputs).  Values are upcast to
float64 exactly.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from .gaunt import layer_paths


def parse_weights(blob: np.ndarray, hp) -> Dict:
    blob = np.asarray(blob, dtype=np.float32)
    C, H, nb, L, S = hp.channels, hp.radial_hidden, hp.n_basis, hp.l_max, hp.n_species
    off = [0]

    def take(shape):
        n = int(np.prod(shape))
        v = blob[off[0]:off[0] + n].astype(np.float64).reshape(shape)
        off[0] += n
        return v

    w = {"W_emb": take((S, C)), "layers": []}
    for t in range(1, hp.n_layers + 1):
        l_in = [0] if t == 1 else list(range(L + 1))
        lay = {"W_up": {l: take((C, C)) for l in l_in},
               "W1": take((nb, H)), "W2": take((H, H))}
        P = len(layer_paths(t, L))
        lay["W3"] = take((H, P * C)).reshape(H, P, C)
        lay["W_down"] = {0: take((C, C * (1 + L)))}
        for l in range(1, L + 1):
            lay["W_down"][l] = take((C, C))
        w["layers"].append(lay)
    w["w_read"] = take((C,))
    w["e0"] = take((S,))
    if off[0] != blob.size:
        raise ValueError(f"weight blob has {blob.size} values, layout needs {off[0]}")
    return w
