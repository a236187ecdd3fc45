"""Host-side logic of the schedule autotuner: table merging and validation of the tuned file (no GPU)."""
import json

import pytest

from paper_1302_7203_amd import binding
from paper_1302_7203_amd.autotune import _merge


def test_merge_keeps_the_last_entry_of_each_run():
    assert _merge([10, 20, 30, 2147483647], [4, 4, 16, 16]) == ([20, 2147483647], [4, 16])
    assert _merge([10, 20], [8, 64]) == ([10, 20], [8, 64])
    assert _merge([5], [1]) == ([5], [1])


def _write(tmp_path, single, batch):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"single": {"n_max": single[0], "lanes": single[1]},
                             "batch": {"n_max": batch[0], "lanes": batch[1]}}))
    return str(p)


def test_read_tuned_accepts_a_valid_table(tmp_path):
    p = _write(tmp_path, ([64, 2147483647], [8, 64]), ([48, 2147483647], [4, 64]))
    t = binding.read_tuned(p)
    assert t["single"] == ([64, 2147483647], [8, 64]) and t["batch"] == ([48, 2147483647], [4, 64])


@pytest.mark.parametrize("single,batch", [
    (([64, 64], [8, 64]), ([48], [4])),          # n_max not increasing
    (([64], [3]), ([48], [4])),                  # lanes not a power of two
    (([64], [8]), ([48], [2])),                  # batch lanes below 4
    (([64], [128]), ([48], [4])),                # more than a wavefront
    (([], []), ([48], [4])),                     # empty
])
def test_read_tuned_rejects_bad_tables(tmp_path, single, batch):
    with pytest.raises(binding.ArrowError):
        binding.read_tuned(_write(tmp_path, single, batch))


def test_missing_file_means_builtin_schedule(tmp_path):
    assert binding.read_tuned(str(tmp_path / "none.json")) is None


def test_committed_table_is_valid():
    t = binding.read_tuned()
    if t is None:
        pytest.skip("no tuned table committed")
    assert t["single"][0][-1] == binding.INT32_MAX and t["batch"][0][-1] == binding.INT32_MAX
