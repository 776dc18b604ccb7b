"""Pins of the CPU U-Net (oracle/unet.py) against brute force, finite differences
and special weight sets whose output has a closed form."""
import numpy as np
import pytest
import torch

from oracle import unet

pytestmark = pytest.mark.filterwarnings("ignore")


def _random_weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout, ks in unet.LAYERS:
        parts.append(rng.normal(0.0, scale * np.sqrt(2.0 / (ks * ks * cin)), cout * ks * ks * cin))
    return np.concatenate(parts)


def _sample(seed, nb, H):
    rng = np.random.default_rng(seed)
    x = np.zeros((nb, H, H, 2))
    x[..., 0] = rng.normal(size=(nb, H, H))
    x[..., 1] = rng.uniform(0.3, 1.9, size=(nb, 1, 1))
    t = rng.normal(size=(nb, H, H))
    return x, t


def test_param_count():
    assert unet.num_params() == sum(cout * ks * ks * cin for cin, cout, ks in unet.LAYERS)
    assert unet.num_params() == 2 * 16 * 9 + 16 * 16 * 9 + 16 * 32 * 9 + 32 * 32 * 9 + 32 * 64 * 9 + 64 * 64 * 9 \
        + 96 * 32 * 9 + 32 * 32 * 9 + 48 * 16 * 9 + 16 * 16 * 9 + 16


def test_weight_layout_brute_force():
    """One 3x3 layer of the oracle against an explicit loop over the flat layout k = (ky*3+kx)*cin+ci."""
    rng = np.random.default_rng(0)
    cin, cout, H = 2, 16, 5
    w0 = rng.normal(size=cout * 9 * cin)
    x = rng.normal(size=(1, H, H, cin))
    k = unet._weights(np.concatenate([w0, np.zeros(unet.num_params() - w0.size)]))[0]
    y = torch.nn.functional.conv2d(torch.as_tensor(x).permute(0, 3, 1, 2), k, padding=1)[0].numpy()
    ref = np.zeros((cout, H, H))
    for co in range(cout):
        for yy in range(H):
            for xx in range(H):
                s = 0.0
                for ky in range(3):
                    for kx in range(3):
                        sy, sx = yy + ky - 1, xx + kx - 1
                        if 0 <= sy < H and 0 <= sx < H:
                            for ci in range(cin):
                                s += w0[co * 9 * cin + (ky * 3 + kx) * cin + ci] * x[0, sy, sx, ci]
                ref[co, yy, xx] = s
    assert np.abs(y - ref).max() < 1e-13


def _centre(w, layer, co, ci):
    cin, cout, ks = unet.LAYERS[layer]
    off = unet.layer_offsets()[layer]
    w[off + co * ks * ks * cin + ((ks // 2) * ks + ks // 2) * cin + ci] = 1.0


def test_skip_path_identity():
    """Weights routing channel 0 through level 1 and the skip s1 only: Net(x) = relu(x0)."""
    w = np.zeros(unet.num_params())
    _centre(w, 0, 0, 0)
    _centre(w, 1, 0, 0)
    _centre(w, 8, 0, 32)   # concat [up(b4) (32 ch), s1 (16 ch)]: s1 channel 0 is input channel 32
    _centre(w, 9, 0, 0)
    _centre(w, 10, 0, 0)
    x, _ = _sample(1, 2, 16)
    y = unet.forward(w, x)
    assert np.abs(y - np.maximum(x[..., 0], 0.0)).max() == 0.0


def test_deep_path_block_average():
    """Weights routing channel 0 through both poolings and upsamplings: 4x4 block averages."""
    w = np.zeros(unet.num_params())
    for layer in range(11):
        _centre(w, layer, 0, 0)  # every concat puts the upsampled path first
    rng = np.random.default_rng(2)
    H = 16
    x = np.zeros((1, H, H, 2))
    x[0, :, :, 0] = rng.uniform(0.0, 1.0, size=(H, H))
    x[0, :, :, 1] = 0.7
    y = unet.forward(w, x)[0]
    blocks = x[0, :, :, 0].reshape(H // 4, 4, H // 4, 4).mean(axis=(1, 3))
    ref = np.kron(blocks, np.ones((4, 4)))
    assert np.abs(y - ref).max() < 1e-15


def test_positive_homogeneity():
    """Bias-free ReLU network: with the alpha channel switched off, Net(c x) = c Net(x) for c > 0."""
    w = _random_weights(3)
    cin, cout, ks = unet.LAYERS[0]
    w0 = w[:cout * ks * ks * cin].reshape(cout, ks * ks, cin)
    w0[:, :, 1] = 0.0
    w[:cout * ks * ks * cin] = w0.ravel()
    x, _ = _sample(4, 1, 16)
    y1 = unet.forward(w, x)
    x2 = x.copy()
    x2[..., 0] *= 3.5
    y2 = unet.forward(w, x2)
    assert np.abs(y2 - 3.5 * y1).max() <= 1e-13 * np.abs(y1).max()


@pytest.mark.parametrize("bf16", [False, True])
def test_gradient_finite_differences(bf16):
    """Central differences of the loss against the autograd gradient, several weights in every layer.
    With bf16 the rounding is piecewise constant, so only the float64 mode is differenced; the bf16
    mode checks that the straight-through gradient equals the float64 gradient at the rounded point."""
    w = _random_weights(5)
    x, t = _sample(6, 2, 16)
    if bf16:
        wr = unet.round_bf16(torch.as_tensor(w)).numpy()
        xr = x.copy()
        xr[..., :] = unet.round_bf16(torch.as_tensor(x)).numpy()
        _, _, g_b = unet.loss_and_grad(wr, xr, t, bf16=True)
        # the forward of bf16 mode at an already-rounded point rounds only the activations,
        # so its gradient differs from the plain one by the rounding of the hidden layers only
        _, _, g_f = unet.loss_and_grad(wr, xr, t, bf16=False)
        assert np.linalg.norm(g_b - g_f) <= 0.05 * np.linalg.norm(g_f)
        return
    L, _, g = unet.loss_and_grad(w, x, t)
    rng = np.random.default_rng(7)
    offs = unet.layer_offsets() + [unet.num_params()]
    for li in range(len(unet.LAYERS)):
        for idx in rng.integers(offs[li], offs[li + 1], size=3):
            hstep = 1e-5 * max(1.0, abs(w[idx]))
            wp, wm = w.copy(), w.copy()
            wp[idx] += hstep
            wm[idx] -= hstep
            fd = (unet.loss(wp, x, t)[0] - unet.loss(wm, x, t)[0]) / (2 * hstep)
            assert abs(fd - g[idx]) <= 1e-6 * max(abs(g[idx]), 1e-3 * np.abs(g).max()), (li, idx, fd, g[idx])


def test_loss_definition():
    """Loss = mean over samples of ||y - t||^2 / ||t||^2; zero at t = y."""
    w = _random_weights(8)
    x, _ = _sample(9, 3, 16)
    y = unet.forward(w, x)
    L, per = unet.loss(w, x, y)
    assert L == 0.0 and np.all(per == 0.0)
    L2, per2 = unet.loss(w, x, 2.0 * y)
    assert np.allclose(per2, 0.25) and abs(L2 - 0.25) < 1e-15


def test_round_bf16_ties_to_even():
    v = torch.tensor([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -(1.0 + 5 * 2.0 ** -9)],
                     dtype=torch.float64)
    r = unet.round_bf16(v).numpy()
    assert r[0] == 1.0                      # tie -> even mantissa
    assert r[1] == 1.0 + 2.0 ** -6          # tie between 1+2^-7 (odd) and 1+2^-6 (even)
    assert r[2] == 1.0                      # below half an ulp
    assert r[3] == -(1.0 + 2.0 ** -7)       # 1+5*2^-9 is 1.25 ulp: nearest


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected update is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(10)
    g = rng.normal(size=50)
    w = rng.normal(size=50)
    w1, m, v = unet.adam_step(w, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(w - w1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # constant gradient: the update stays lr * sign(g) up to eps at every step
    wk, mk, vk = w.copy(), np.zeros(50), np.zeros(50)
    for k in range(1, 6):
        wn, mk, vk = unet.adam_step(wk, mk, vk, g, k, 1e-3)
        assert np.allclose(wk - wn, 1e-3 * np.sign(g), rtol=1e-6, atol=0)
        wk = wn


def test_apply_scale_invariance():
    """z(c r) = c z(r): the residual is normalised before the network."""
    w = _random_weights(11)
    rng = np.random.default_rng(12)
    r = rng.normal(size=(15, 15))
    z1 = unet.apply(w, r, 1.2, 16)
    z2 = unet.apply(w, 7.0 * r, 1.2, 16)
    assert np.abs(z2 - 7.0 * z1).max() <= 1e-13 * np.abs(z2).max()
    x = unet.net_input(r, 16, 1.2)
    assert abs(np.mean(x[:15, :15, 0] ** 2) - 1.0) < 1e-14 and np.all(x[15, :, 0] == 0) and np.all(x[..., 1] == 1.2)


def test_fp32_evaluation_is_the_same_network():
    # the FP32 CPU evaluation (the scale the GPU's fp32-operand gates are set against) computes
    # the same network: its distance from the FP64 forward is FP32 rounding only, and the
    # distance grows when the weights and inputs are rounded further (to bf16)
    rng = np.random.default_rng(5)
    w = np.concatenate([rng.normal(0.0, np.sqrt(2.0 / (ks * ks * cin)), cout * ks * ks * cin)
                        for cin, cout, ks in unet.LAYERS]).astype(np.float32)
    x = rng.normal(size=(2, 32, 32, 2)).astype(np.float32)
    ref = unet.forward(w.astype(np.float64), x)
    y32 = unet.forward_fp32(w, x)
    e = np.linalg.norm(y32 - ref) / np.linalg.norm(ref)
    assert 1e-9 < e < 3e-6, e
    eb = np.linalg.norm(unet.forward(w.astype(np.float64), x, bf16=True) - ref) / np.linalg.norm(ref)
    assert eb > 100 * e
