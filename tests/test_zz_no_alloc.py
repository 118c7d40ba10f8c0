"""gl_mlp_infer_noalloc, the inference entry point that allocates nothing,
against gl_mlp_infer through the C-ABI: bitwise the same outputs on two calls
in a row, the second with a smaller input (the fixed scratch array keeps the
first call's contents, which must not leak into the second), an input larger
than one pass of the array, and the refusal of a network too wide for it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_07999_amd as g
    g.lib()
    return g


def _inputs(n, seed):
    g = np.random.default_rng(seed)
    lo = np.array([1.0, 0.0, 0.0, 0.0, 0.0])
    hi = np.array([3.0, 4.2, 10.0, 0.2, 1.0])
    return g.uniform(lo, hi, size=(n, 5)).astype(np.float32)


def test_noalloc_inference_equals_workspace_inference(gl):
    import torch
    net = gl.MLP(5, 256, 3, 2, max_batch=1024, max_samples=16, seed=21)
    net.set_scaling([1, 0, 0, 0, 0], [3, 4.2, 10, 0.2, 1], [0.3, -0.2], [1.5, 0.7])
    net.set_output_power(0, [3.0, 2.0])
    for n, seed in ((5000, 1), (37, 2), (1, 3), (2048, 4)):
        X = torch.from_numpy(_inputs(n, seed)).cuda()
        want = net.infer(X).cpu().numpy()
        got = net.infer_noalloc(X).cpu().numpy()
        print("n=%d: max |noalloc - infer| = %.1e" % (n, np.abs(got - want).max()))
        assert got.shape == want.shape == (n, 2)
        assert np.array_equal(got, want)
        assert np.isfinite(got).all() and np.abs(got).max() > 0


def test_noalloc_refuses_a_network_too_wide(gl):
    import torch
    wide = gl.MLP(5, 20000, 1, 2, max_batch=1, max_samples=1, seed=1)
    X = torch.from_numpy(_inputs(3, 5)).cuda()
    with pytest.raises(gl.GlasmaError) as e:
        wide.infer_noalloc(X)
    assert e.value.status == gl.GL_EINVAL and "too wide" in str(e.value)
