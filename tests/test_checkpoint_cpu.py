"""Checkpoint files of a PDFB state (host side): round trip bit for bit with
the dtypes kept, refusal of a file written for another plan configuration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
fhs = pytest.importorskip("paper_2003_07358_amd")
from paper_2003_07358_amd import checkpoint  # noqa: E402


def test_round_trip_is_bitwise(tmp_path):
    plan = fhs.Plan(40, 36, 6, 2, 2, 1, 4, 4, 2)
    s = plan.sizes
    rng = np.random.default_rng(3)
    state = {"x": torch.from_numpy(rng.standard_normal(s["n_x"]).astype(np.float32)),
             "p": torch.from_numpy(rng.standard_normal(s["n_p"]).astype(np.float32)),
             "theta_bar": torch.from_numpy(rng.uniform(0.5, 1.0, s["n_theta_bar"])),
             "xi": torch.tensor([np.inf, 1e-3], dtype=torch.float64)}
    path = tmp_path / "state.npz"
    checkpoint.save(path, plan, **state)
    back = checkpoint.load(path, plan, device="cpu")
    assert sorted(back) == sorted(state)
    for k, v in state.items():
        assert back[k].dtype == v.dtype and torch.equal(back[k], v), k


def test_other_plan_is_refused(tmp_path):
    plan = fhs.Plan(40, 36, 6, 2, 2, 1, 4, 4, 2)
    path = tmp_path / "state.npz"
    checkpoint.save(path, plan, x=torch.zeros(plan.sizes["n_x"]))
    other = fhs.Plan(40, 36, 6, 2, 2, 1, 6, 6, 2)
    with pytest.raises(fhs.FhsError):
        checkpoint.load(path, other, device="cpu")
