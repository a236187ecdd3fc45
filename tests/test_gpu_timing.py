"""Stage timing of single solves: events stamped by the kernels' own dispatches,
kept for the two most recent timed calls (read one while the next is queued)."""
import numpy as np
import pytest

from paper_1302_7203_amd import binding, workloads as W

pytestmark = pytest.mark.gpu


def test_timing_of_two_calls_in_turn():
    import torch
    dev = torch.device("cuda", 0)
    pr = W.uniform_arrow(1024, np.random.default_rng(7))
    d = torch.from_numpy(pr.d).to(dev)
    z = torch.from_numpy(pr.z).to(dev)
    ref = binding.arrow_eig(d, z, pr.scalar)
    binding.set_option(binding.OPT_TIMING, 1)
    try:
        outs, seen = [], []
        for s in range(4):
            outs.append(binding.arrow_eig(d, z, pr.scalar))
            if s > 0:
                seen.append(binding.timing_of(1))   # the previous call, this one still queued
        seen.append(binding.timing_of(0))
        assert np.allclose(binding.last_timing(), seen[-1])
        with pytest.raises(binding.ArrowError):
            binding.timing_of(2)
    finally:
        binding.set_option(binding.OPT_TIMING, 0)
    torch.cuda.synchronize()
    for st in seen:
        st = np.array(st)
        assert np.all(np.isfinite(st)) and np.all(st >= 0.0), st
        assert st[2] > 0.0 and st[4] > 0.0, st      # the root and vector kernels' own durations
        assert st.sum() < 1e3, st
    # timing changes nothing in the results
    for o in outs:
        assert torch.equal(o.lam, ref.lam) and torch.equal(o.V, ref.V)
