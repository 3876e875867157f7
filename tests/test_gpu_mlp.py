"""The rank-predictor network on the GPU against the FP64 reference network.

* Forward pass: equal to the reference evaluated with the same (BF16-rounded)
  weights, up to FP32 accumulation (1e-5 relative).
* Gradients: equal to the reference's with the same weights to 1e-3 relative
  (FP32 accumulation), and within 1e-2 of the reference with the unrounded
  FP32 master weights (the BF16 rounding of the weights).
* Training with Adam lowers the loss on a synthetic regression task.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import mlp as omlp
    from paper_1703_09085_amd import hm

    return torch, hm, omlp, hm.Context()


def params64(hm, vec):
    return {k: np.asarray(v, dtype=np.float64) for k, v in hm.mlp_unpack(vec.astype(np.float64)).items()}


def test_forward_and_gradients(env):
    torch, hm, omlp, ctx = env
    net = hm.MLP(ctx, seed=5)
    master, working = net.weights()
    rng = np.random.default_rng(2)
    X = rng.standard_normal((300, 8)).astype(np.float32)
    t = rng.standard_normal(300).astype(np.float32)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    y = net.predict(Xd).cpu().numpy()
    pw = params64(hm, working)
    yr, _ = omlp.forward(pw, X.astype(np.float64))
    assert np.max(np.abs(y - yr)) <= 1e-5 * max(1.0, np.max(np.abs(yr)))
    # the working copy is the BF16 rounding of the master weights
    mats = np.r_[0:512, 576:4672, 4736:4800]
    assert np.array_equal(working[mats], omlp.to_bf16(master[mats]).astype(np.float32))
    g, loss = net.gradient(Xd, td)
    gr = omlp.gradients(pw, X.astype(np.float64), t.astype(np.float64))
    gvec = np.concatenate([np.ravel(gr[k]) for k, _ in hm.MLP_LAYOUT])
    assert np.linalg.norm(g - gvec) <= 1e-3 * np.linalg.norm(gvec)
    assert loss == pytest.approx(omlp.loss(pw, X.astype(np.float64), t.astype(np.float64)), rel=1e-5)
    gm = omlp.gradients(params64(hm, master), X.astype(np.float64), t.astype(np.float64))
    gmvec = np.concatenate([np.ravel(gm[k]) for k, _ in hm.MLP_LAYOUT])
    assert np.linalg.norm(g - gmvec) <= 1e-2 * np.linalg.norm(gmvec)


def test_training_lowers_the_loss(env):
    torch, hm, omlp, ctx = env
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (4096, 8)).astype(np.float32)
    t = (np.abs(X[:, 0]) * 3 + np.maximum(X[:, 1], 0) * 2 - X[:, 2] * X[:, 3]).astype(np.float32)
    net = hm.MLP(ctx, seed=1)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    losses = net.train(Xd, td, epochs=40, batch=256, lr=3e-3)
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.1 * losses[0]
    master, working = net.weights()
    yr, _ = omlp.forward(params64(hm, working), X.astype(np.float64))
    assert 0.5 * np.mean((yr - t) ** 2) < 0.1 * losses[0]
