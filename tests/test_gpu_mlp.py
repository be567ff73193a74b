"""The surrogate network's BF16 matrix-core kernels against the FP64 oracle.

Two references: the FP64 oracle itself (BF16 tolerance), and the same
products with every matrix-core operand rounded to BF16 first and summed in
FP64 (then only FP32 accumulation and FP32 GELU differ)."""
import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu

DIMS = [6, 256, 256, 256, 7]


def bf16(a):
    """Round to BF16 (nearest even) and back, in float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, dims, X):
    layers = M.split(np.asarray(params, dtype=np.float64), dims)
    A = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        Z = bf16(A) @ bf16(W) + b
        cache.append((A, Z))
        A = M.gelu(Z) if l < len(layers) - 1 else Z
    return A, cache


def gradients_bf16(params, dims, X, Y):
    layers = M.split(np.asarray(params, dtype=np.float64), dims)
    Yh, cache = forward_bf16(params, dims, X)
    dA = 2.0 * (Yh - Y) / Yh.size
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        Ain, Z = cache[l]
        dZ = dA if l == len(layers) - 1 else dA * M.gelu_grad(Z)
        grads.append((bf16(Ain).T @ bf16(dZ), dZ.sum(axis=0)))
        dA = bf16(dZ) @ bf16(W).T
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def setup(batch=300, seed=0):
    import torch
    from paper_2506_05362_amd import mlp
    rng = np.random.default_rng(seed)
    p = M.init_params(DIMS, seed=seed) + rng.normal(0, 0.02, M.n_params(DIMS))
    p = p.astype(np.float32).astype(np.float64)
    X = rng.normal(size=(batch, DIMS[0]))
    Y = rng.normal(size=(batch, DIMS[-1]))
    net = mlp.Net(DIMS, max_batch=512)
    net.set_params(p)
    return net, p, X, Y, torch


def test_forward_matches_oracle():
    net, p, X, Y, torch = setup()
    y = net.forward(torch.tensor(X, dtype=torch.float32)).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(p, DIMS, X)
    emu, _ = forward_bf16(p, DIMS, X)
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 3e-2 * scale
    # activations are rounded to BF16 from an FP32 GELU on the GPU and an FP64 one in the
    # emulation: a value on a rounding boundary flips one operand by a BF16 ulp
    assert np.linalg.norm(y - emu) <= 2e-4 * np.linalg.norm(emu)
    assert np.abs(y - emu).max() <= 3e-3 * scale


def test_forward_large_batch_chunks_and_ragged_tail():
    net, p, _, _, torch = setup()
    rng = np.random.default_rng(4)
    X = rng.normal(size=(1291, DIMS[0]))  # several max_batch chunks and a ragged tail
    y = net.forward(torch.tensor(X, dtype=torch.float32)).cpu().numpy()
    emu, _ = forward_bf16(p, DIMS, X)
    assert np.linalg.norm(y - emu) <= 2e-4 * np.linalg.norm(emu)
    assert np.abs(y - emu).max() <= 3e-3 * np.abs(emu).max()


def test_fused_inference_matches_emulation_and_layer_path():
    """The fused two-kernel inference path (weights in LDS) against the BF16
    emulation and against the layer-by-layer kernels, over several max_batch
    chunks, a ragged tail and a tile that is only partly filled."""
    net, p, _, _, torch = setup()
    rng = np.random.default_rng(5)
    X = rng.normal(size=(1291, DIMS[0]))
    xt = torch.tensor(X, dtype=torch.float32)
    net.set_inference(True)
    yf = net.forward(xt).cpu().numpy()
    net.set_inference(False)
    yl = net.forward(xt).cpu().numpy()
    emu, _ = forward_bf16(p, DIMS, X)
    for y in (yf, yl):
        assert np.linalg.norm(y - emu) <= 2e-4 * np.linalg.norm(emu)
        assert np.abs(y - emu).max() <= 3e-3 * np.abs(emu).max()
    assert np.linalg.norm(yf - yl) <= 2e-4 * np.linalg.norm(yl)
    for m in (1, 17, 64, 65):  # short and partial tiles
        net.set_inference(True)
        ym = net.forward(xt[:m]).cpu().numpy()
        assert np.linalg.norm(ym - emu[:m]) <= 2e-4 * np.linalg.norm(emu[:m])


@pytest.mark.parametrize("din,dout", [(12, 16), (16, 1)])
def test_fused_inference_wide_inputs_and_outputs(din, dout):
    """The fused path's other instantiation (9 to 16 inputs) and the output
    widths at its limits, against the BF16 emulation over a ragged batch."""
    import torch
    from paper_2506_05362_amd import mlp
    dims = [din, 256, 256, 256, dout]
    rng = np.random.default_rng(din)
    p = (M.init_params(dims, seed=din) + rng.normal(0, 0.02, M.n_params(dims))).astype(np.float32).astype(np.float64)
    net = mlp.Net(dims, max_batch=512)
    net.set_params(p)
    X = rng.normal(size=(700, din))
    net.set_inference(True)
    y = net.forward(torch.tensor(X, dtype=torch.float32)).cpu().numpy()
    emu, _ = forward_bf16(p, dims, X)
    assert np.linalg.norm(y - emu) <= 2e-4 * np.linalg.norm(emu)
    assert np.abs(y - emu).max() <= 3e-3 * np.abs(emu).max()


def test_fused_inference_unsupported_shape():
    import torch
    from paper_2506_05362_amd import mlp
    net = mlp.Net([5, 32, 32, 32, 3], max_batch=64)
    with pytest.raises(mlp.MLPError):
        net.set_inference(True)
    net.set_inference(False)
    assert net.forward(torch.zeros((3, 5))).shape == (3, 3)


def test_gradients_match_oracle():
    net, p, X, Y, torch = setup(batch=257)
    loss, g = net.gradients(torch.tensor(X, dtype=torch.float32), torch.tensor(Y, dtype=torch.float32))
    assert loss == pytest.approx(M.loss(p, DIMS, X, Y), rel=2e-2)
    ref = M.gradients(p, DIMS, X, Y)
    emu = gradients_bf16(p, DIMS, X, Y)
    g = g.astype(np.float64)
    assert np.linalg.norm(g - ref) <= 5e-2 * np.linalg.norm(ref)
    assert np.linalg.norm(g - emu) <= 2e-3 * np.linalg.norm(emu)
    assert np.abs(g - emu).max() <= 2e-3 * np.abs(emu).max()


def test_adam_step_matches_oracle_update():
    net, p, X, Y, torch = setup(batch=128)
    xt, yt = torch.tensor(X, dtype=torch.float32, device="cuda"), torch.tensor(Y, dtype=torch.float32, device="cuda")
    _, g = net.gradients(xt, yt)
    net.train_step(xt, yt, lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    expect, _, _ = M.adam_step(p, g.astype(np.float64), np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    assert np.abs(p1 - expect).max() <= 1e-6 + 1e-5 * 1e-3


def test_adam_weight_decay_matches_oracle_update():
    net, p, X, Y, torch = setup(batch=128)
    net.set_adam(weight_decay=0.05)
    xt, yt = torch.tensor(X, dtype=torch.float32, device="cuda"), torch.tensor(Y, dtype=torch.float32, device="cuda")
    _, g = net.gradients(xt, yt)
    net.train_step(xt, yt, lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    expect, _, _ = M.adam_step(p, g.astype(np.float64), np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3,
                               weight_decay=0.05)
    assert np.abs(p1 - expect).max() <= 1e-6 + 1e-5 * 1e-3


def test_training_reduces_loss_on_a_smooth_target():
    import torch
    from paper_2506_05362_amd import mlp
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, size=(2048, 6))
    Y = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2], np.cos(X[:, 3]), X[:, 4] ** 2,
                  X[:, 5], X[:, 0] * X[:, 5], np.tanh(X[:, 1]), X.sum(axis=1) / 3], axis=1)
    net = mlp.Net(DIMS, max_batch=512)
    net.set_params(M.init_params(DIMS, seed=1).astype(np.float32))
    xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    yt = torch.tensor(Y, dtype=torch.float32, device="cuda")
    first = None
    for it in range(300):
        s = (it * 512) % 2048
        loss = net.train_step(xt[s:s + 512], yt[s:s + 512], lr=1e-3)
        first = loss if first is None else first
    assert loss < 0.05 * first
