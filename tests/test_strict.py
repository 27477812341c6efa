"""require_converged on hand-made stats records (host only): channels that
stopped at the iteration cap or on d^T A d <= 0 raise NotConverged, the other
reasons (tolerance met, r^T s = 0, b = 0) do not."""
import numpy as np
import pytest
import torch

from paper_1511_03296_amd import NotConverged, read_stats, require_converged
from paper_1511_03296_amd.solver import _STATS_DTYPE


def stats_of(reasons):
    rec = np.zeros(len(reasons), dtype=_STATS_DTYPE)
    rec["reason"] = reasons
    rec["iters"] = 7
    rec["rel_residual"] = [1e-3 * (i + 1) for i in range(len(reasons))]
    return torch.from_numpy(np.frombuffer(rec.tobytes(), dtype=np.uint8).copy())


def test_reads_back_what_was_written():
    st = stats_of([1, 2, 5])
    rec = read_stats(st)
    assert rec["reason"].tolist() == [1, 2, 5] and rec["iters"].tolist() == [7, 7, 7]


@pytest.mark.parametrize("reasons", [[1], [1, 3, 5], [5, 5]])
def test_met_tolerances_pass(reasons):
    require_converged(stats_of(reasons))


@pytest.mark.parametrize("reasons,bad", [([2], 1), ([1, 4, 1], 1), ([2, 4, 1, 2], 3)])
def test_missed_tolerances_raise(reasons, bad):
    with pytest.raises(NotConverged) as e:
        require_converged(stats_of(reasons), "adjoint solve")
    msg = str(e.value)
    assert msg.startswith("adjoint solve") and f"({bad} of {len(reasons)} channels)" in msg
