"""Checkpoint files: a round trip keeps W, the state bytes and t bit for bit,
and a file for another problem is refused (no device needed)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")
from paper_2410_19844_amd import checkpoint as C  # noqa: E402


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_round_trip_is_bitwise(tmp_path, prec):
    pl = S.Plan(4, 2, 11, prec, device="cpu")
    g = torch.Generator().manual_seed(3)
    W = torch.randn((pl.N, pl.rank), generator=g, dtype=torch.float64).to(pl.wdtype)
    state = torch.randint(0, 256, (pl.state_bytes,), generator=g, dtype=torch.uint8)
    f = str(tmp_path / "ck.npz")
    C.save(f, pl, W, state, 17)
    W2, st2, t = C.load(f, pl)
    assert t == 17 and W2.dtype == pl.wdtype and torch.equal(W2.view(torch.uint8), W.view(torch.uint8))
    assert torch.equal(st2, state)
    with np.load(f, allow_pickle=False) as z:      # plain arrays only
        assert set(z.files) == {"format", "shape", "precision", "t", "W", "state"}


def test_other_problem_is_refused(tmp_path):
    pl = S.Plan(4, 2, 11, "fp32", device="cpu")
    W = torch.zeros((pl.N, pl.rank), dtype=torch.float32)
    f = str(tmp_path / "ck.npz")
    C.save(f, pl, W, torch.zeros(pl.state_bytes, dtype=torch.uint8), 1)
    for other in (S.Plan(4, 2, 12, "fp32", device="cpu"), S.Plan(4, 2, 11, "fp64", device="cpu")):
        with pytest.raises(ValueError):
            C.load(f, other)
