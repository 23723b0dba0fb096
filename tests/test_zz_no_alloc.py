"""mpip_evaluate_noalloc against mpip_evaluate through the C ABI.

The no-alloc entry point runs the evaluation of mpip_evaluate with the
library's static device workspace instead of a caller workspace.  Two calls
in a row on one model (the second with fewer atoms, so it runs over what the
first left in the static array) must give the outputs of mpip_evaluate on the
same inputs; the kernels and their reduction orders are the same, so the
results are compared bit for bit.  A system whose workspace exceeds the
static array is rejected on the host before anything runs."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def M(torch):
    import paper_2509_21694_amd as m
    return m


def _outputs(torch, n, dev):
    return {"energy": torch.full((1,), float("nan"), dtype=torch.float64, device=dev),
            "forces": torch.full((n, 3), float("nan"), dtype=torch.float64, device=dev),
            "virial": torch.full((3, 3), float("nan"), dtype=torch.float64, device=dev),
            "atom_energy": torch.full((n,), float("nan"), dtype=torch.float64, device=dev)}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_matches_evaluate(torch, M, prec):
    hp = W.HP_MPDP
    model = M.Model(hp, W.make_weights(hp, W.WEIGHT_SEEDS["mpdp"]))
    dev = torch.device("cuda", 0)
    for n_side, seed in ((12, 611), (7, 612)):          # 1,728 atoms, then 343
        s = W.bulk_system(n_side, seed, seed + 1)
        assert model.workspace_bytes(s.n_atoms, 2, prec, M.estimate_edges(s.n_atoms, s.cell, hp.r_cut)) \
            <= M.NOALLOC_SCRATCH_BYTES
        pos = torch.tensor(s.positions, dtype=torch.float64, device=dev)
        sp = torch.tensor(s.species, dtype=torch.int32, device=dev)
        print(f"noalloc {prec}: {s.n_atoms} atoms", flush=True)
        ref = model.evaluate(pos, sp, s.cell, s.pbc, K=2, precision=prec, atom_energy=True)
        o = model.evaluate_noalloc(pos, sp, s.cell, s.pbc, _outputs(torch, s.n_atoms, dev), K=2, precision=prec)
        torch.cuda.synchronize()
        for k in ("energy", "forces", "virial", "atom_energy"):
            a, b = o[k].cpu().numpy(), ref[k].cpu().numpy()
            assert np.all(np.isfinite(a)), k
            assert np.array_equal(a, b), (k, float(np.abs(a - b).max()))


def test_noalloc_rejects_oversized_system(torch, M):
    hp = W.HP_BULK
    model = M.Model(hp, W.make_weights(hp, W.WEIGHT_SEEDS["bulk1m"]))
    s = W.bulk_system(30, 613, 614)                      # 27,000 atoms at C = 128: beyond the static array
    dev = torch.device("cuda", 0)
    pos = torch.tensor(s.positions, dtype=torch.float64, device=dev)
    sp = torch.tensor(s.species, dtype=torch.int32, device=dev)
    o = _outputs(torch, s.n_atoms, dev)
    with pytest.raises(M.MpipError) as ei:
        model.evaluate_noalloc(pos, sp, s.cell, s.pbc, o, K=2, precision="bf16")
    assert ei.value.status == M.ECAPACITY
    torch.cuda.synchronize()
    assert torch.isnan(o["energy"]).all()                # nothing ran
