"""Proposal-network kernels against the FP64 oracle: covariance packing,
forward, gradients (FP32 and BF16 GEMM operands), Adam steps, and a short
training run."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bartlett as ob
from oracle import mlp as om
from paper_2604_19723_amd import bartlett as bb
from paper_2604_19723_amd import workload as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def normwise(a, b):
    return np.max(np.abs(np.asarray(a, np.float64) - b)) / max(np.max(np.abs(b)), 1e-30)


def make(prec, dims, B, seed=0, max_batch=None):
    rng = np.random.default_rng(seed)
    params = om.init_params(dims[0], dims[1], len(dims) - 2, dims[-1], rng)
    net = bb.ba_mlp_create(dims[0], dims[1], len(dims) - 2, dims[-1], max_batch or B, prec, seed)
    bb.ba_mlp_set_weights(net, bb.mlp_list_to_params(params))
    # the device holds FP32 master weights: compare against those values
    params = bb.mlp_params_to_list(bb.ba_mlp_get_weights(net).astype(np.float64), net.dims)
    X = rng.standard_normal((B, dims[0])).astype(np.float32)
    T = rng.standard_normal((B, dims[-1])).astype(np.float32)
    mask = (rng.uniform(size=(B, dims[-1])) > 0.25).astype(np.float32)
    return net, params, X, T, mask


def test_pack_matches_oracle():
    ts = wl.config5(6)
    with bb.plan_for(ts) as plan:
        Y = torch.from_numpy(ts.y_c64()).to(DEV)
        R = torch.empty((6, 64, 64), dtype=torch.complex64, device=DEV)
        bb.ba_covariance(plan, 6, 256, Y, R)
        X = torch.empty((6, 4096), dtype=torch.float32, device=DEV)
        bb.ba_pack_covariance(64, 6, R, X)
        Rh = R.cpu().numpy().astype(np.complex128)
        Xh = X.cpu().numpy()
    for b in range(6):
        np.testing.assert_allclose(Xh[b], om.pack_covariance(Rh[b]), rtol=2e-6, atol=2e-6)


@pytest.mark.parametrize("dims,B", [((96, 64, 64, 4), 50), ((4096, 512, 512, 512, 4), 64)])
def test_forward_and_gradients_f32(dims, B):
    net, params, X, T, mask = make(bb.BA_PREC_F32, dims, B)
    Xd, Td, Md = (torch.from_numpy(a).to(DEV) for a in (X, T, mask))
    Y = torch.empty((B, dims[-1]), dtype=torch.float32, device=DEV)
    bb.ba_mlp_forward(net, B, Xd, Y)
    g = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    bb.ba_mlp_gradients(net, B, Xd, Td, Md, g, loss)
    torch.cuda.synchronize()
    Yr, cache = om.forward(params, X.astype(np.float64))
    Lr, dY = om.mse_loss(Yr, T.astype(np.float64), mask.astype(np.float64))
    gr = om.backward(params, cache, dY)
    assert normwise(Y.cpu().numpy(), Yr) <= 1e-5
    assert abs(loss.item() - Lr) <= 1e-5 * abs(Lr)
    gg = bb.mlp_params_to_list(g.cpu().numpy(), net.dims)
    for (gW, gb), (rW, rb) in zip(gg, gr):
        assert normwise(gW, rW) <= 1e-4
        assert normwise(gb, rb) <= 1e-4
    net.close()


def test_forward_and_gradients_bf16():
    dims, B = (4096, 512, 512, 512, 4), 64
    net, params, X, T, mask = make(bb.BA_PREC_BF16, dims, B, seed=1)
    Xd, Td, Md = (torch.from_numpy(a).to(DEV) for a in (X, T, mask))
    Y = torch.empty((B, 4), dtype=torch.float32, device=DEV)
    bb.ba_mlp_forward(net, B, Xd, Y)
    g = torch.empty(net.n_params, dtype=torch.float32, device=DEV)
    bb.ba_mlp_gradients(net, B, Xd, Td, Md, g)
    torch.cuda.synchronize()
    Yr, cache = om.forward(params, X.astype(np.float64))
    gr = om.backward(params, cache, om.mse_loss(Yr, T.astype(np.float64), mask.astype(np.float64))[1])
    e_y = normwise(Y.cpu().numpy(), Yr)
    # the same network with its GEMM operands rounded to BF16 in the oracle
    Yb, _ = om.forward(params, X.astype(np.float64), round_fn=om.bf16_round)
    print("BF16 forward: vs FP64 %.2e, vs FP64-with-BF16-operands %.2e" % (e_y, normwise(Y.cpu().numpy(), Yb)))
    assert e_y <= 2e-2
    assert normwise(Y.cpu().numpy(), Yb) <= 2e-3
    gg = bb.mlp_params_to_list(g.cpu().numpy(), net.dims)
    for (gW, gb), (rW, rb) in zip(gg, gr):
        assert normwise(gW, rW) <= 5e-2
        assert normwise(gb, rb) <= 5e-2
    net.close()


def test_adam_steps_match_oracle():
    dims, B = (96, 64, 64, 4), 40
    net, params, X, T, mask = make(bb.BA_PREC_F32, dims, B, seed=2)
    Xd, Td, Md = (torch.from_numpy(a).to(DEV) for a in (X, T, mask))
    opt = om.Adam(params, lr=1e-3)
    cur = params
    for _ in range(3):
        bb.ba_mlp_train_step(net, B, Xd, Td, Md, 1e-3)
        Yr, cache = om.forward(cur, X.astype(np.float64))
        gr = om.backward(cur, cache, om.mse_loss(Yr, T.astype(np.float64), mask.astype(np.float64))[1])
        cur = opt.step(cur, gr)
    torch.cuda.synchronize()
    got = bb.ba_mlp_get_weights(net).astype(np.float64)
    ref = bb.mlp_list_to_params(cur)
    start = bb.mlp_list_to_params(params)
    d_got, d_ref = got - start, ref - start
    close = np.abs(d_got - d_ref) <= 1e-4 * 1e-3 * 3 + 1e-6 * np.abs(ref)
    # elements whose gradient is at rounding level can flip their Adam direction
    assert np.mean(close) > 0.999, np.mean(close)
    net.close()


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    dims = (32, 64, 2, 4)
    teacher = om.init_params(32, 16, 1, 4, rng)
    X = rng.standard_normal((512, 32))
    T, _ = om.forward(teacher, X)
    net = bb.ba_mlp_create(32, 64, 2, 4, 512, bb.BA_PREC_BF16, 7)
    Xd = torch.from_numpy(X.astype(np.float32)).to(DEV)
    Td = torch.from_numpy(T.astype(np.float32)).to(DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    bb.ba_mlp_train_step(net, 512, Xd, Td, None, 3e-3, loss)
    first = loss.item()
    for _ in range(300):
        bb.ba_mlp_train_step(net, 512, Xd, Td, None, 3e-3, loss)
    last = loss.item()
    print("loss %.4e -> %.4e" % (first, last))
    assert last < 0.1 * first
    net.close()


def test_mlp_argument_errors():
    net = bb.ba_mlp_create(8, 8, 1, 2, 16, bb.BA_PREC_F32, 0)
    X = torch.zeros((32, 8), device=DEV)
    T = torch.zeros((32, 2), device=DEV)
    with pytest.raises(bb.BartlettError):
        bb.ba_mlp_train_step(net, 32, X, T, None, 1e-3)       # above max_batch
    with pytest.raises(bb.BartlettError):
        bb.ba_mlp_train_step(net, 8, X, T, None, -1.0)
    with pytest.raises(ValueError):
        bb.ba_mlp_set_weights(net, np.zeros(3))
    net.close()
