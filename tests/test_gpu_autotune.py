"""The autotuner on the device: a quick run writes a valid table that handles accept, and a
handle with that table still solves to the oracle's accuracy."""
import numpy as np
import pytest

import oracle
from paper_1302_7203_amd import workloads as W
from parity import assert_close

pytestmark = pytest.mark.gpu


def test_quick_autotune_writes_a_usable_table(tmp_path, oracle_lib):
    import torch
    from paper_1302_7203_amd import autotune, binding
    out = str(tmp_path / "schedule.json")
    try:
        assert autotune.main(["--quick", "--out", out]) == 0
        t = binding.read_tuned(out)
        h = binding.handle(0)
        binding.apply_tuned(h, out)
        pr = W.uniform_arrow(256, np.random.default_rng(4))
        r = binding.arrow_eig(torch.from_numpy(pr.d).cuda(), torch.from_numpy(pr.z).cuda(), pr.scalar)
        torch.cuda.synchronize()
        ref = oracle.arrow_eig(pr.d, pr.z, pr.scalar)
        assert_close(r.lam.cpu().numpy(), ref.lam, "values")
        assert_close(r.V.cpu().numpy(), ref.vec, "vectors")
        assert t["single"][0][-1] == binding.INT32_MAX
    finally:
        h = binding.handle(0)
        binding.set_lanes_table(binding.SCHEDULE_SINGLE, [], [], h=h)
        binding.set_lanes_table(binding.SCHEDULE_BATCH, [], [], h=h)
        binding.apply_tuned(h)
