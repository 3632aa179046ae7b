"""GPU tests of the learned residual corrector through the C ABI, against the FP64 oracle.

Tolerances: the 64 x 64 layer runs on BF16 MFMA (weights and activations rounded to BF16,
unit roundoff 2^-8, FP32 accumulation).  The oracle is given the same BF16-rounded W2, so the
remaining differences come from rounding the hidden activations and the layer-2 error
signal: per-tensor relative L2 errors are bounded by a few unit roundoffs, stated below as
2e-2 for the first layer (two rounded products away from the loss) and 1e-2 elsewhere.  The
kernel's FP32 reference mode (fst_mlp_grad_fp32: the 64 x 64 layer in FP32, nothing rounded
to BF16) matches the oracle's gradients to 1e-5 per tensor."""
import numpy as np
import pytest

import datagen
from oracle import mlp
from oracle.reconstruct import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
fst = pytest.importorskip("paper_1907_05884_amd.binding")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def D(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


def _params(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    for k in p:
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    flat = mlp.flatten(p).astype(np.float32)
    flat[256:4352] = bf16_round(flat[256:4352])       # W2 as the MFMA sees it
    return flat


def test_gradients_match_oracle(dev):
    flat = _params(3)
    lo, hi = (0.0, 0.0, 0.0), (4.0, 1.0, 1.0)
    n, B = 5000, 700                                   # batch not a multiple of the 64-point tile
    rng = np.random.default_rng(4)
    pts = (np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * rng.random((n, 3))).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    idx = rng.integers(0, n, B).astype(np.int32)
    c = fst.fst_corrector_from_params(lo, hi, flat, 1.0)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    g = fst.fst_mlp_grad(c, x, y, z, D(t, dev), D(idx, dev)).cpu().numpy().astype(np.float64)
    xi = 2.0 * (pts[idx].astype(np.float64) - np.asarray(lo)) / (np.asarray(hi) - np.asarray(lo)) - 1.0
    loss, gr = mlp.loss_and_grads(mlp.unflatten(flat.astype(np.float64)), xi, t[idx].astype(np.float64))
    ref = mlp.flatten(gr)
    seg = {"W1": (0, 192, 2e-2), "b1": (192, 256, 2e-2), "W2": (256, 4352, 1e-2), "b2": (4352, 4416, 1e-2),
           "W3": (4416, 4480, 1e-2), "b3": (4480, 4481, 1e-2)}
    for name, (a, b, tol) in seg.items():
        assert rel_l2(g[a:b], ref[a:b]) <= tol, name
    assert g[4481] / B == pytest.approx(loss, rel=1e-2)


def test_apply_matches_oracle_forward(dev):
    flat = _params(5)
    flat = bf16_round(flat)                             # stored parameters are BF16 values
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    n = 10007
    pts = np.random.default_rng(6).uniform(-1, 1, (n, 3)).astype(np.float32)
    c = fst.fst_corrector_from_params(lo, hi, flat, 2.5)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    base = np.random.default_rng(7).standard_normal(n).astype(np.float32)
    out = fst.fst_corrector_apply(c, x, y, z, D(base, dev)).cpu().numpy()
    yref, _ = mlp.forward(mlp.unflatten(flat.astype(np.float64)), pts.astype(np.float64))
    assert rel_l2(out - base, 2.5 * yref) <= 1e-2
    assert c.stored_bytes() == 2 * 4481 + 4


def test_training_reduces_loss_and_held_out_error(dev):
    # a smooth model plus a sharp planar front that the model cannot represent
    rank, degree = (4, 4, 4), (7, 7, 7)
    core, coefs = datagen.random_model_parts(8, rank, degree)
    gm = fst.fst_model_from_parts((-1,) * 3, (1,) * 3, rank, degree, core, coefs)
    rng = np.random.default_rng(9)
    n = 60000
    pts = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    base = fst.fst_eval(gm, x, y, z).cpu().numpy()
    front = np.tanh((pts @ np.array([0.48, 0.6, 0.64]) - 0.1) / 0.05).astype(np.float32)
    v = base + front
    ntr = 50000
    tp = fst.make_train_params(steps=1500, batch=2048, lr=3e-3, seed=2)
    c = fst.fst_corrector_train(gm, x[:ntr].contiguous(), y[:ntr].contiguous(), z[:ntr].contiguous(),
                                D(v[:ntr], dev), tp)
    losses = c.losses()
    assert losses[-1] < 0.2 * losses[0]
    xh, yh, zh = x[ntr:].contiguous(), y[ntr:].contiguous(), z[ntr:].contiguous()
    plain = fst.fst_eval(gm, xh, yh, zh).cpu().numpy()
    corr = fst.fst_eval_corrected(gm, c, xh, yh, zh).cpu().numpy()
    e_plain = rel_l2(plain, v[ntr:])
    e_corr = rel_l2(corr, v[ntr:])
    assert e_corr < 0.5 * e_plain, (e_plain, e_corr)


def test_adam_steps_match_oracle(dev):
    # three Adam steps from the same parameters on the same counter-drawn minibatches
    from oracle.sampler import batch_indices
    flat = bf16_round(_params(11))
    rank, degree = (3, 3, 3), (5, 5, 5)
    core, coefs = datagen.random_model_parts(12, rank, degree)
    gm = fst.fst_model_from_parts((-1,) * 3, (1,) * 3, rank, degree, core, coefs)
    n = 4000
    pts = np.random.default_rng(13).uniform(-1, 1, (n, 3)).astype(np.float32)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    f = fst.fst_eval(gm, x, y, z).cpu().numpy().astype(np.float64)
    v = (f + np.sin(4 * pts[:, 0]) * pts[:, 1]).astype(np.float32)
    lr = 1e-3
    tp = fst.make_train_params(steps=3, batch=512, lr=lr, seed=7, init_params=flat)
    c = fst.fst_corrector_train(gm, x, y, z, D(v, dev), tp)
    gpu_after, sd = c.params()
    # oracle: the same scaled residual target, the same batches, FP64 Adam
    e = v.astype(np.float64) - f
    t = e / e.std()
    params = mlp.unflatten(flat.astype(np.float64))
    opt = mlp.Adam(params, lr=lr)
    for s in range(3):
        idx = batch_indices(7, s, 512, n)
        _, g = mlp.loss_and_grads(params, pts[idx].astype(np.float64), t[idx])
        params = opt.step(params, g)
    ref_after = mlp.flatten(params)
    d_gpu = gpu_after.astype(np.float64) - flat
    d_ref = ref_after - flat
    # the stored parameters are BF16-rounded after training: compare updates above that rounding
    big = np.abs(d_ref) > 4 * np.abs(flat) * 2.0 ** -8
    assert big.sum() > 100
    assert rel_l2(d_gpu[big], d_ref[big]) <= 0.1
    assert sd == pytest.approx(e.std(), rel=1e-4)


def test_gradients_fp32_mode_match_oracle(dev):
    # the reference mode of the training kernel (64 x 64 layer in FP32, no BF16 rounding of W2 or
    # of the activations) against the FP64 oracle: FP32 arithmetic throughout, per-point terms
    # summed over 64-point tiles and then over the tiles in FP32, so each gradient entry carries
    # a few units of 2^-24 of the sum of its terms' magnitudes
    rng = np.random.default_rng(13)
    p = mlp.init_params(13)
    for k in p:
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    flat = mlp.flatten(p).astype(np.float32)
    lo, hi = (0.0, 0.0, 0.0), (4.0, 1.0, 1.0)
    n, B = 5000, 700
    pts = (np.asarray(lo) + (np.asarray(hi) - np.asarray(lo)) * rng.random((n, 3))).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    idx = rng.integers(0, n, B).astype(np.int32)
    c = fst.fst_corrector_from_params(lo, hi, flat, 1.0)
    x, y, z = [D(pts[:, k], dev) for k in range(3)]
    g = fst.fst_mlp_grad(c, x, y, z, D(t, dev), D(idx, dev), fp32=True).cpu().numpy().astype(np.float64)
    xi = 2.0 * (pts[idx].astype(np.float64) - np.asarray(lo)) / (np.asarray(hi) - np.asarray(lo)) - 1.0
    loss, gr = mlp.loss_and_grads(mlp.unflatten(flat.astype(np.float64)), xi, t[idx].astype(np.float64))
    ref = mlp.flatten(gr)
    for name, (a, b) in {"W1": (0, 192), "b1": (192, 256), "W2": (256, 4352), "b2": (4352, 4416),
                         "W3": (4416, 4480), "b3": (4480, 4481)}.items():
        err = rel_l2(g[a:b], ref[a:b])
        print(f"fp32 mode {name}: rel-L2 {err:.2e}", flush=True)
        assert err <= 1e-5, name
    assert g[4481] / B == pytest.approx(loss, rel=1e-5)
