"""helm_apply_oras_noalloc (the allocation-free one-level ORAS application)
against helm_apply_oras, through the C ABI, on two calls in a row (the second
smaller), on both levels and both precisions, plus its refusals."""
import numpy as np
import pytest

import inputs
from oracle.operator import fit_weights

pytestmark = pytest.mark.gpu

WO = fit_weights()
W = {k: getattr(WO, k) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")}


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_noalloc_oras_matches_the_allocating_entry_point(prec, tol):
    import torch
    from paper_2103_14921_amd import helm
    shape, h, f = (28, 26, 24), 25.0, 10.0
    c = inputs.velocity_thrust_belt(*shape, h=h, q=100.0)
    S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2,
                    precision=prec)
    dev = torch.device("cuda:0")
    for level, nrhs, seed in ((0, 6, 1), (0, 3, 2), (1, 5, 3), (1, 2, 4)):  # each level: a call, then a smaller one
        n = S.n if level == 0 else S.nc
        say("noalloc", prec, "level", level, "nrhs", nrhs)
        R = inputs.random_field((nrhs, n), seed=seed)
        ref = S.apply_oras(R, level=level)
        Rd = torch.from_numpy(R).to(dev)
        Zd = torch.full((nrhs, n), float("nan"), dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        S.apply_oras_noalloc(Rd, Zd, level=level)
        torch.cuda.synchronize()
        Z = Zd.cpu().numpy()
        assert np.all(np.isfinite(Z))
        assert rel(Z, ref) <= tol, (level, nrhs, rel(Z, ref))
        assert np.array_equal(Rd.cpu().numpy(), R)
    S.close()


def test_noalloc_oras_refuses_host_memory_and_oversized_batches():
    import torch
    from paper_2103_14921_amd import helm
    shape, h, f = (28, 26, 24), 25.0, 10.0
    c = inputs.velocity_thrust_belt(*shape, h=h)
    S = helm.Solver(shape, h, c, f, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=1)
    say("noalloc refusals")
    R = inputs.random_field((2, S.n), seed=5)
    with pytest.raises(helm.HelmError) as e:
        S.apply_oras_noalloc(R, np.empty_like(R))
    assert e.value.code == helm.HELM_EINVAL and "device memory" in str(e.value)
    dev = torch.device("cuda:0")
    big = torch.zeros((256, S.n), dtype=torch.complex128, device=dev)  # 256 x 17472 nodes: > 64 MiB of staging
    with pytest.raises(helm.HelmError) as e:
        S.apply_oras_noalloc(big, torch.empty_like(big))
    assert e.value.code == helm.HELM_EINVAL and "limit" in str(e.value)
    assert "limit" in S.last_error()
    S.close()
