"""Allocator bridge of concord_create: the handle's device workspace comes from the
caller's allocator (PyTorch's caching allocator through TorchAllocator), gives the
same iterates as hipMalloc'd workspace, is returned in full on destroy, and an
allocator that returns NULL is reported as ENOMEM with every earlier block returned."""
import numpy as np
import pytest

import datagen
from tests.gpu_common import max_abs_diff

pytestmark = pytest.mark.gpu


def _data(p, n):
    import torch
    w = datagen.make_workload("c2_obs_p20000", p=p, n=n)
    return torch.from_numpy(w.X.astype(np.float32)).cuda(), w.lam2


@pytest.mark.parametrize("variant", ["cov", "obs"])
def test_bridge_matches_hipmalloc_and_returns_everything(variant):
    import torch
    from paper_1710_10769_amd import Solver, TorchAllocator
    p, n = 700, 300
    X, lam2 = _data(p, n)
    print(f"[case] allocator bridge {variant} fp32 p={p} n={n}", flush=True)
    outs = []
    for mode in ("hip", "torch"):
        alloc = None if mode == "hip" else TorchAllocator(torch.cuda.current_device())
        before = torch.cuda.memory_allocated()
        s = Solver(p, n, variant=variant, precision="fp32", allocator=alloc)
        s.set_data(X)
        if alloc is not None:
            assert alloc.n_alloc > 0 and torch.cuda.memory_allocated() > before
        infos = [s.step(0.12, lam2) for _ in range(5)]
        outs.append(([(i.tau, i.F, i.nnz) for i in infos], s.get_omega_scipy()))
        s.close()
        if alloc is not None:
            assert not alloc.live and alloc.n_free == alloc.n_alloc
            assert torch.cuda.memory_allocated() == before
    assert outs[0][0] == outs[1][0]
    assert max_abs_diff(outs[0][1], outs[1][1]) == 0.0


@pytest.mark.parametrize("fail_after", [0, 3, 12])
def test_null_allocation_is_enomem(fail_after):
    import torch
    from paper_1710_10769_amd import ConcordError, Solver, TorchAllocator
    from paper_1710_10769_amd._lib import ENOMEM
    print(f"[case] allocator returns NULL after {fail_after} blocks", flush=True)
    alloc = TorchAllocator(torch.cuda.current_device(), fail_after=fail_after)
    with pytest.raises(ConcordError) as e:
        Solver(500, 200, variant="cov", precision="fp32", allocator=alloc)
    assert e.value.code == ENOMEM
    assert alloc.n_alloc == fail_after and not alloc.live


def test_regrowth_failure_is_enomem_and_handle_survives():
    """A dense candidate set needs more capacity mid-step; a refused regrowth fails the
    step with ENOMEM and leaves the iterate as it was."""
    import torch
    from paper_1710_10769_amd import ConcordError, Solver, TorchAllocator
    from paper_1710_10769_amd._lib import ENOMEM
    p, n = 300, 120
    X, lam2 = _data(p, n)
    print(f"[case] regrowth refused cov fp32 p={p}", flush=True)
    alloc = TorchAllocator(torch.cuda.current_device())
    s = Solver(p, n, variant="cov", precision="fp32", allocator=alloc)
    s.set_data(X)
    before = s.get_omega_scipy()
    alloc.fail_after = alloc.n_alloc   # refuse every further block
    with pytest.raises(ConcordError) as e:
        for _ in range(4):
            s.step(0.01, lam2)          # lambda1 this small grows the candidate set
    assert e.value.code == ENOMEM
    assert s.iterations == 0 and max_abs_diff(s.get_omega_scipy(), before) == 0.0
    s.close()
    assert not alloc.live
