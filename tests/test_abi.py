"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
agrees with the generator on the weight count, rejects bad arguments on the
host, and its independently derived coupling tensors (Wigner 3j + complex to
real change of basis) equal the oracle's quadrature tensors."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle.gaunt import coupling_tensor as oracle_cg, natural

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2509_21694_amd as M
    return M


def test_exports_match_header():
    M = _lib()
    header = open(os.path.join(ROOT, "include", "mpip.h")).read()
    declared = set(re.findall(r"\b(mpip_[a-z_]+)\s*\(", header))
    assert declared == set(M.EXPORTED)
    for name in declared:
        assert hasattr(M.lib, name)
    cdll = ctypes.CDLL(M.LIB_PATH)
    for name in declared:
        getattr(cdll, name)


@pytest.mark.parametrize("hp", [W.HP_SMALL, W.HP_MPDP, W.HP_BULK, W.HP_BATCH])
def test_weight_count(hp):
    assert _lib().weights_count(hp) == W.weights_count(hp)


def test_invalid_hparams_rejected():
    M = _lib()
    import dataclasses
    for bad in [dict(l_max=3), dict(channels=48), dict(n_layers=0), dict(n_basis=6)]:
        hp = dataclasses.replace(W.HP_SMALL, **bad)
        assert M.weights_count(hp) == 0


def test_coupling_tensors_match_oracle():
    M = _lib()
    n = 0
    for l1 in range(3):
        for l2 in range(3):
            for l3 in range(3):
                if natural(l1, l2, l3):
                    assert np.allclose(M.coupling_tensor(l1, l2, l3), oracle_cg(l1, l2, l3), atol=1e-13)
                    n += 1
                else:
                    with pytest.raises(M.MpipError):
                        M.coupling_tensor(l1, l2, l3)
    assert n == 11


def test_host_validation_without_gpu():
    M = _lib()
    # null model -> EINVAL before any device work
    s = M.SystemC()
    st = M.lib.mpip_evaluate(None, ctypes.byref(s), 0, 1, None, None, 0, 0, None)
    assert st == M.EINVAL
    # triclinic cells are rejected on the host by the GPU neighbour search
    s.n_atoms = 4
    s.n_owned = 4
    s.positions = 16
    s.species = 16
    for k, v in enumerate([10, 1, 0, 0, 10, 0, 0, 0, 10]):
        s.cell[k] = v
    for k in range(3):
        s.pbc[k] = 1
    ne = ctypes.c_int64()
    st = M.lib.mpip_neighbor_list(ctypes.byref(s), 5.0, None, ctypes.c_void_p(16), 1 << 20, 0,
                                  None, None, None, ctypes.byref(ne))
    assert st == M.EUNSUPPORTED
