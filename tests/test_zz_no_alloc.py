"""arrow_eig_noalloc (the entry point that allocates nothing: its workspace is a
static device array) against arrow_eig, through the C ABI: two calls in a row,
the second with a smaller input, each bitwise equal to arrow_eig's result on the
same input and within 1e-13 of the oracle; orders above the scratch's maximum
are refused."""
import numpy as np
import pytest

import near_zero_cases as NZ
import oracle
from paper_1302_7203_amd import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu


def test_noalloc_matches_arrow_eig_twice(oracle_lib):
    import torch
    from paper_1302_7203_amd import binding
    assert torch.cuda.is_available()
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(2024)
    # a graded problem with clusters (remedies, the repair launch) and a smaller one
    # whose eigenvalue nearest 0 takes Remark 1 (the exact sum in LDS)
    big = W.graded_arrow(3001, rng, clusters=8, cluster_size=8)
    _, d, z, a = NZ.arrow_cases()[-1]
    small = W.Problem(W.KIND_ARROW, d.size + 1, d, z, a)
    for name, pr in (("graded n=3001", big), ("near zero n=301", small)):
        print(f"arrow_eig_noalloc vs arrow_eig: {name}", flush=True)
        d = torch.from_numpy(pr.d).to(dev)
        z = torch.from_numpy(pr.z).to(dev)
        a = binding.arrow_eig(d, z, pr.scalar, pairs=True)
        b = binding.arrow_eig(d, z, pr.scalar, pairs=True, noalloc=True)
        torch.cuda.synchronize(dev)
        for x, y in ((a.lam, b.lam), (a.V, b.V), (a.shift, b.shift), (a.mu, b.mu), (a.info, b.info)):
            assert torch.equal(x, y), name
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        if pr is small:
            assert int(b.info[int(np.argmin(np.abs(ref.lam)))]) & 8   # Remark 1 ran, in the scratch too
        assert_close(b.lam.cpu().numpy(), ref.lam, f"{name} lambda")
        assert_close(b.V.cpu().numpy(), ref.vec, f"{name} V")


def test_noalloc_refuses_orders_above_its_scratch():
    import torch
    from paper_1302_7203_amd import binding
    dev = torch.device("cuda", 0)
    n = binding.NOALLOC_N_MAX + 1
    d = torch.zeros(n - 1, dtype=torch.float64, device=dev)
    with pytest.raises(binding.ArrowError):
        binding.arrow_eig(d, d, 0.0, vectors=False, noalloc=True)
