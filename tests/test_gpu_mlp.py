"""GPU MLP kernels against the float64 reference.

Tolerances: the kernels compute in FP32 (unit roundoff u = 2^-24 ~ 6e-8).
A forward pass sums 4 then 64 products per unit, so its error is a few times
64 u relative to the magnitude of the terms: |y_gpu - y_ref| <= 1e-4 (1 + |y|)
has two orders of margin.  A gradient entry is a sum over B rows of products
of activations that each went through about 140 rounded operations (4-term
and 64-term dot products forward, a 64-term one backward), so by the forward
error bound of sums and dot products every entry is within (B + 300) u of
its own magnitude (the oracle's grad_magnitude: the same chain rule over
absolute values).  That bound holds while rounding flips no ReLU mask, so the
inputs keep every pre-activation at least 1e-3 of its terms' magnitude away
from zero (rows are selected by the oracle's relu_margin).
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2203_13512_amd as kc  # noqa: E402


def _setup(seed, rows):
    r = np.random.default_rng(seed)
    p = M.init_params(seed) + r.normal(0, 0.02, M.NPARAMS)
    x = r.normal(0, 1, (rows, 4))
    t = r.normal(0, 2, rows)
    dev = torch.device("cuda:0")
    P = torch.tensor(p, dtype=torch.float32, device=dev)
    X = torch.tensor(x, dtype=torch.float32, device=dev)
    T = torch.tensor(t, dtype=torch.float32, device=dev)
    # the reference sees the same FP32-rounded inputs
    return p.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64), \
        t.astype(np.float32).astype(np.float64), P, X, T


@pytest.mark.parametrize("rows", [1, 63, 1000, 70001])
def test_forward_matches_reference(rows):
    p, x, t, P, X, T = _setup(rows, rows)
    y = kc.mlp_forward(P, X).cpu().numpy().astype(np.float64)
    want = M.forward(p, x)
    assert np.all(np.abs(y - want) <= 1e-4 * (1 + np.abs(want)))


@pytest.mark.parametrize("rows", [1, 256, 4097, 20000])
def test_gradient_and_loss_match_reference(rows):
    p, x, t, P, X, T = _setup(7 + rows, 2 * rows + 64)
    keep = np.flatnonzero(M.relu_margin(p, x) > 1e-3)[:rows]
    assert len(keep) == rows
    x, t = x[keep], t[keep]
    X, T = X[torch.from_numpy(keep).to(X.device)].contiguous(), T[torch.from_numpy(keep).to(T.device)].contiguous()
    loss, grad = kc.mlp_train_step(P, X, T)
    L, g = M.loss_and_grad(p, x, t)
    assert abs(float(loss.item()) - L) <= 1e-4 * (1 + L)
    gg = grad.cpu().numpy().astype(np.float64)
    bound = (rows + 300) * 2.0 ** -24 * M.grad_magnitude(p, x, t)
    assert np.all(np.abs(gg - g) <= bound + 1e-30), np.max(np.abs(gg - g) / (bound + 1e-30))


def test_adam_step_matches_reference():
    p, x, t, P, X, T = _setup(3, 512)
    m = torch.zeros(kc.MLP_NPARAMS, device=P.device)
    v = torch.zeros(kc.MLP_NPARAMS, device=P.device)
    mr, vr, pr = np.zeros(M.NPARAMS), np.zeros(M.NPARAMS), p.copy()
    for step in range(1, 4):
        _, g = M.loss_and_grad(pr, x, t)
        pr, mr, vr = M.adam_step(pr, g, mr, vr, step, 1e-2)
        kc.mlp_train_step(P, X, T, m, v, t=step, lr=1e-2)
    got = P.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - pr) <= 2e-4 * (1 + np.abs(pr)))


def test_training_throughput():
    """Rows per second of a full training step (forward, backward, Adam) on a
    minibatch of 4096 rows, reported; a step must take well under a
    millisecond per thousand rows."""
    import time
    p, x, t, P, X, T = _setup(11, 4096)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    ws = torch.empty(kc.mlp_workspace_size(4096), dtype=torch.uint8, device=P.device)
    for step in range(1, 4):
        kc.mlp_train_step(P, X, T, m, v, t=step, lr=1e-3, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 50
    for step in range(4, 4 + steps):
        kc.mlp_train_step(P, X, T, m, v, t=step, lr=1e-3, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    print(f"mlp training step, 4096 rows: {dt * 1e3:.3f} ms ({4096 / dt:.3e} rows/s)", flush=True)
    assert dt < 4e-3


def test_training_reduces_the_loss():
    r = np.random.default_rng(9)
    x = r.normal(0, 1, (4096, 4))
    t = np.log1p(np.exp(x @ np.array([1.0, -0.5, 2.0, 0.25])))  # smooth target
    dev = torch.device("cuda:0")
    P = torch.tensor(M.init_params(4), dtype=torch.float32, device=dev)
    X = torch.tensor(x, dtype=torch.float32, device=dev)
    T = torch.tensor(t, dtype=torch.float32, device=dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    first = None
    for step in range(1, 301):
        loss, _ = kc.mlp_train_step(P, X, T, m, v, t=step, lr=3e-3)
        if first is None:
            first = float(loss.item())
    last = float(kc.mlp_train_step(P, X, T)[0].item())
    assert last < 0.05 * first
