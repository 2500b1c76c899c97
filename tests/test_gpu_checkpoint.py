"""Resume from a checkpoint on the grouped (serving) path, whose sums run in a
fixed order: the steps after the resume match the uninterrupted run bit for
bit (W, the Adam moments and the losses)."""
import math

import pytest

from workloads import gaussian

torch = pytest.importorskip("torch")
S = pytest.importorskip("paper_2410_19844_amd")
from paper_2410_19844_amd import checkpoint as C  # noqa: E402

pytestmark = pytest.mark.gpu


def test_resume_is_bitwise_on_the_grouped_path(tmp_path):
    dev = torch.device("cuda")
    shapes = [(4, 2), (5, 3)]
    plans, Ws, sts, ps = [], [], [], []
    for q, (n, d) in enumerate(shapes):
        pl = S.Plan(n, d, 2 * math.comb(n + d, d), "fp32")
        W0 = torch.tensor(gaussian((pl.N, 3), 40 + q), dtype=torch.float32, device=dev)
        z = torch.zeros(pl.M, dtype=torch.float64, device=dev)
        _, _, p = S.Plan(n, d, 3, "fp32").loss_grad(W0, z, grad=False, want_r=True, exact=True)
        plans.append(pl)
        Ws.append(torch.tensor(gaussian((pl.N, pl.rank), 50 + q, 0.3), dtype=torch.float32, device=dev))
        sts.append(pl.new_state())
        ps.append(p.contiguous())
    adam = S.Adam(lr=3e-2)
    losses = torch.empty(len(plans), dtype=torch.float64, device=dev)

    def run(t0, t1, Ws, sts):
        out = []
        for t in range(t0, t1):
            S.step_batch(plans, Ws, sts, [t] * len(plans), ps, adam, losses)
            out.append(losses.clone())
        return out

    run(1, 21, Ws, sts)
    files = [str(tmp_path / f"ck{q}.npz") for q in range(len(plans))]
    for f, pl, W, st in zip(files, plans, Ws, sts):
        C.save(f, pl, W, st, 20)
    L_a = run(21, 31, Ws, sts)
    restored = [C.load(f, pl) for f, pl in zip(files, plans)]
    assert all(t == 20 for _, _, t in restored)
    W_b = [w for w, _, _ in restored]
    st_b = [s for _, s, _ in restored]
    L_b = run(21, 31, W_b, st_b)
    for a, b in zip(L_a, L_b):
        assert torch.equal(a, b)
    for wa, wb, sa, sb in zip(Ws, W_b, sts, st_b):
        assert torch.equal(wa, wb)
        assert torch.equal(sa, sb)
