"""The learned warm start against the zero start (small, fast version of the experiment):
a network trained on solver-generated solutions at n = 32 gives held-out starts whose
(minimal-residual scaled) initial residual is below 1, fewer GMRES iterations than the zero
start on average, and warm-started solves that still reach the FP64 tolerance.  The WKB start
without the network is measured beside it, and both gains are printed."""
import numpy as np
import pytest

from paper_2204_00326_amd import ls, warmstart

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_learned_start_reduces_iterations():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 32
    data = warmstart.generate(range(0, 96), n, angles_per_contrast=2, tol=1e-8)
    net = ls.NeuralOperator(n, width=16, modes=8, layers=4, batch_max=16, seed=1, bf16=True)
    hist = warmstart.train(net, data, epochs=40, batch=16, lr=3e-3)
    print("loss", hist[0], hist[-1], flush=True)
    rows = warmstart.evaluate(net, range(100000, 100016), n, hodlr_rank=0)
    z = np.array([r["its_zero"] for r in rows])
    w = np.array([r["its_warm"] for r in rows])
    b = np.array([r["its_wkb"] for r in rows])
    r0 = np.array([r["warm_relres0"] for r in rows])
    print("its zero", z.tolist(), "learned", w.tolist(), "wkb only", b.tolist(), flush=True)
    print("relres0", np.round(r0, 3).tolist(), "saved", 1 - w.sum() / z.sum(), "wkb only", 1 - b.sum() / z.sum(),
          flush=True)
    assert hist[-1] < 0.5 * hist[0]
    assert np.all(r0 <= 1.0) and np.median(r0) < 0.9
    assert w.mean() < z.mean()
    assert all(r["status_warm"] == "CONVERGED" and r["relres_warm"] <= 1.01e-8 for r in rows)
