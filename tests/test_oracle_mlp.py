"""Pins of the FP64 reference network (oracle/mlp.py).

* Gradients agree with central finite differences of the loss in every
  parameter group (the chain rule against the definition of the derivative).
* A forward pass with hand-chosen weights has a closed form.
* BF16 rounding of known values (round to nearest, ties to even).
"""
import numpy as np
import pytest

pytest.importorskip("oracle")
from oracle import mlp  # noqa: E402


def random_params(rng, scale=0.5):
    return {k: (rng.standard_normal(s) * scale if s else np.float64(rng.standard_normal() * scale))
            for k, s in mlp.SHAPES.items()}


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = random_params(rng)
    X = rng.standard_normal((17, 8))
    t = rng.standard_normal(17)
    g = mlp.gradients(p, X, t)
    for name, shape in mlp.SHAPES.items():
        size = int(np.prod(shape)) if shape else 1
        for idx in rng.choice(size, size=min(size, 6), replace=False):
            fd = mlp.finite_difference(p, X, t, name, int(idx))
            an = g[name].reshape(-1)[idx] if shape else g[name]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_forward_closed_form():
    """W1 copies the 8 features into the first 8 hidden units (scaled by 2),
    W2 is the identity, w3 sums: y = 2 sum_i relu(x_i) + b3."""
    p = {k: np.zeros(s) if s else np.float64(0.0) for k, s in mlp.SHAPES.items()}
    for i in range(8):
        p["W1"][i, i] = 2.0
    p["W2"] = np.eye(64)
    p["w3"][:] = 1.0
    p["b3"] = np.float64(0.25)
    X = np.array([[1.0, -2.0, 3.0, 0.5, -0.5, 0.0, 4.0, -1.0]])
    y, _ = mlp.forward(p, X)
    assert y[0] == pytest.approx(2 * (1.0 + 3.0 + 0.5 + 4.0) + 0.25, abs=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 1.0 + 2.0 ** -9])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, -2.5, 1.0])
    assert np.array_equal(mlp.to_bf16(vals), want)
