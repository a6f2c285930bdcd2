"""The allocation-free forward pass of the perceptron (feast_mlp_forward_noalloc) against the
workspace entry point (feast_mlp_forward) through the C ABI: the same kernels on the same inputs, so
the outputs must agree bit for bit.  Two calls in a row, the second with a smaller batch (the static
scratch keeps the first call's activations), and a size above the scratch's limit rejected."""
import numpy as np
import pytest

from oracle import mlp
from tests.gpu_common import device

pytestmark = pytest.mark.gpu


def _f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device())


@pytest.mark.parametrize("half", [True, False])
def test_noalloc_forward_matches_workspace_forward(half):
    import paper_1404_2891_amd as fm
    g = np.random.default_rng(77 + int(half))
    n_in, hidden = 19, 256
    P = mlp.flatten(mlp.init_params(g, n_in, hidden))
    net = fm.MLP(P, n_in=n_in, hidden=hidden, half=half, max_batch=1024, device=device())
    params = _f32(P)
    for batch in (1000, 37):   # the second call is smaller than the first
        X = _f32(g.standard_normal((batch, n_in)) * 2.0 + 0.5)
        want = net.forward(X).cpu().numpy()
        got = fm.binding.mlp_forward_noalloc(params, X, n_in, hidden, half=half).cpu().numpy()
        assert got.shape == want.shape
        assert np.array_equal(got, want), float(np.max(np.abs(got - want)))
    net.close()


def test_noalloc_forward_with_standardization():
    """Moments passed explicitly equal the ones the workspace path measured (fit_standardization):
    the workspace path is given them by measuring them on a set whose moments are exactly those."""
    import paper_1404_2891_amd as fm
    g = np.random.default_rng(91)
    n_in, hidden = 19, 256
    P = mlp.flatten(mlp.init_params(g, n_in, hidden))
    net = fm.MLP(P, n_in=n_in, hidden=hidden, half=True, max_batch=512, device=device())
    # two rows m - s and m + s per column have mean m and population deviation s exactly
    m = np.round(g.uniform(-2, 2, n_in) * 8) / 8
    s = 2.0 ** np.round(g.uniform(-1, 2, n_in))
    net.fit_standardization(_f32(np.stack([m - s, m + s])))
    X = _f32(g.standard_normal((300, n_in)) * 2.0 + 0.5)
    want = net.forward(X).cpu().numpy()
    got = fm.binding.mlp_forward_noalloc(_f32(P), X, n_in, hidden, half=True, x_mean=_f32(m),
                                         x_scale=_f32(s)).cpu().numpy()
    assert np.array_equal(got, want), float(np.max(np.abs(got - want)))
    net.close()


def test_noalloc_rejects_batches_beyond_the_scratch():
    import paper_1404_2891_amd as fm
    lim = int(fm.binding.lib().feast_mlp_noalloc_max_elems())
    n_in, hidden = 3, 256
    batch = lim // hidden + 1
    P = _f32(np.zeros(fm.binding.lib().feast_mlp_param_count(n_in, hidden)))
    X = _f32(np.zeros((batch, n_in)))
    with pytest.raises(fm.FeastError) as e:
        fm.binding.mlp_forward_noalloc(P, X, n_in, hidden)
    assert e.value.code == -8
