"""The surrogate's hand-written BF16 MFMA kernels against the FP64 network
oracle: forward outputs, gradients of one backward pass (the oracle rounds to
BF16 where the device stores BF16, so the remaining differences are FP32
accumulation order and rare one-ulp BF16 rounding differences), and a short
training run that must reduce the loss."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


SHAPE = (5, 256, 3, 2)
LO = np.array([1.0, 0.0, 0.0, 0.0, 0.0])
HI = np.array([3.0, 4.2, 10.0, 0.2, 1.0])
MU = np.array([0.5, -1.0])
SD = np.array([2.0, 3.0])


def _data(n, seed):
    g = np.random.default_rng(seed)
    X = g.uniform(LO, HI, size=(n, 5))
    Y = np.stack([np.sin(2 * X[:, 4]) * X[:, 0] + 0.1 * X[:, 2], np.cos(X[:, 1]) * X[:, 4]], axis=1)
    return X, Y


@pytest.mark.parametrize("n", [1, 70, 256, 1000])
def test_forward_matches_oracle(gl, n):
    net = gl.MLP(*SHAPE, max_batch=1024, max_samples=4096, seed=3)
    net.set_scaling(LO, HI, MU, SD)
    p = net.params().astype(np.float64)
    X, _ = _data(n, 5)
    got = net.infer(X.astype(np.float32)).cpu().numpy()
    Zs, _ = M.forward(p, M.scale_inputs(X.astype(np.float32), LO.astype(np.float32), HI.astype(np.float32)), SHAPE,
                      bf16=True)
    want = Zs[-1] * SD + MU
    assert np.abs(got - want).max() < 2e-2 * np.abs(want).max()
    assert np.corrcoef(got.ravel(), want.ravel())[0, 1] > 0.9999


def test_gradients_match_oracle(gl):
    net = gl.MLP(*SHAPE, max_batch=512, max_samples=4096, seed=4)
    net.set_scaling(LO, HI, MU, SD)
    p = net.params().astype(np.float64)
    X, Y = _data(384, 6)
    g, loss = net.grads(X.astype(np.float32), Y.astype(np.float32))
    Xs = M.scale_inputs(X.astype(np.float32), LO.astype(np.float32), HI.astype(np.float32))
    Ys = (Y.astype(np.float32) - MU) / SD
    lo_, go = M.loss_and_grads(p, Xs, Ys, SHAPE, bf16=True)
    assert abs(loss - lo_) < 1e-3 * lo_
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    cos = g @ go / (np.linalg.norm(g) * np.linalg.norm(go))
    assert rel < 2e-2 and cos > 0.9998, (rel, cos)
    # per layer, including the tiny input and output layers
    L, din, dout = M.dims(*SHAPE)
    off = 0
    for l in range(L):
        k = din[l] * dout[l]
        a, b = g[off:off + k], go[off:off + k]
        assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b) + 1e-12
        off += k


def test_training_reduces_loss_and_fits(gl):
    net = gl.MLP(*SHAPE, max_batch=1024, max_samples=65536, seed=7)
    X, Y = _data(32768, 8)
    net.set_scaling(LO, HI, Y.mean(0), Y.std(0))
    losses = net.train(X.astype(np.float32), Y.astype(np.float32), epochs=12, batch=512, lr=2e-3, seed=1)
    assert losses[-1] < 0.05 * losses[0], losses
    Xt, Yt = _data(4096, 9)
    pred = net.infer(Xt.astype(np.float32)).cpu().numpy()
    err = np.abs(pred - Yt).max(axis=0) / np.abs(Yt).max(axis=0)
    assert np.all(err < 0.1), err


def test_forward_and_gradients_match_oracle_elementwise(gl):
    """Every output and every gradient element within a bound derived from
    BF16 rounding: the device and the oracle round the same operands to BF16,
    but their FP32 and FP64 accumulations can land on the two sides of a BF16
    rounding boundary, which changes an operand by one BF16 ulp (2^-8
    relative).  An element then moves by at most 2^-8 times the sum of the
    magnitudes of its terms (oracle.grad_scales, oracle.output_scales), so
    |device - oracle| <= 2^-8 * scale per element, plus an FP32 floor."""
    n = 384
    net = gl.MLP(*SHAPE, max_batch=512, max_samples=4096, seed=11)
    net.set_scaling(LO, HI, MU, SD)
    p = net.params().astype(np.float64)
    X, Y = _data(n, 12)
    Xs = M.scale_inputs(X.astype(np.float32), LO.astype(np.float32), HI.astype(np.float32))
    # forward
    got = net.infer(X.astype(np.float32)).cpu().numpy()
    Zs, _ = M.forward(p, Xs, SHAPE, bf16=True)
    want = Zs[-1] * SD + MU
    scale = M.output_scales(p, Xs, SHAPE, bf16=True) * SD
    rf = np.abs(got - want) / (scale + 1e-30)
    # gradients
    g, loss = net.grads(X.astype(np.float32), Y.astype(np.float32))
    Ys = (Y.astype(np.float32) - MU) / SD
    _, go = M.loss_and_grads(p, Xs, Ys, SHAPE, bf16=True)
    A = M.grad_scales(p, Xs, Ys, SHAPE, bf16=True)
    rg = np.abs(g - go) / (A + 1e-30)
    L, din, dout = M.dims(*SHAPE)
    off, parts = 0, []
    for l in range(L):
        k = din[l] * dout[l]
        parts.append(("W%d" % (l + 1), rg[off:off + k]))
        off += k
    for l in range(L):
        parts.append(("b%d" % (l + 1), rg[off:off + dout[l]]))
        off += dout[l]
    print("forward: max |dev - orc| / scale = %.2e" % rf.max())
    for name, r in parts:
        print("%s: max |dev - orc| / scale = %.2e (median %.1e)" % (name, r.max(), np.median(r)))
    u = 2.0 ** -8
    assert rf.max() < u
    assert rg.max() < u
