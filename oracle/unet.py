"""FP64 CPU U-Net of the learned preconditioner -- TEST INFRASTRUCTURE ONLY.

The learned preconditioner is not part of Duo & Zhang's method; it is the
network that feeds the flexible PCG of the GPU library.  This module is its
plain definition in PyTorch CPU float64 ops (conv2d, average pooling,
nearest upsampling, concatenation, ReLU) with gradients by autograd and
Adam (Kingma & Ba, Algorithm 1) written out in numpy.  It shares no code
with the HIP path.

Architecture (bias-free 3x3 convolutions, ReLU after all but the last):
  level 1 @ H:   2 -> 16 -> 16         (skip s1)
  pool 2x2, level 2 @ H/2: 16 -> 32 -> 32  (skip s2)
  pool 2x2, level 3 @ H/4: 32 -> 64 -> 64
  up x2 (nearest), concat [up, s2] = 96 -> 32 -> 32
  up x2 (nearest), concat [up, s1] = 48 -> 16 -> 16
  1x1 convolution 16 -> 1
Weights are one flat vector, layer after layer, each layer [cout][k] with
k = (ky*ks + kx)*cin + ci; the tap (ky, kx) reads the input at
(y + ky - ks//2, x + kx - ks//2) (cross-correlation, zero padding).
Samples are NHWC: x[b, y, x, c], c = 0 the scaled residual, c = 1 alpha.

``bf16=True`` rounds every convolution's input activations and weights to
bfloat16 (through float32, round to nearest even) before the product, as
the production GEMMs do; gradients pass straight through the rounding.
"""
import numpy as np
import torch
import torch.nn.functional as F

LAYERS = [(2, 16, 3), (16, 16, 3), (16, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3),
          (96, 32, 3), (32, 32, 3), (48, 16, 3), (16, 16, 3), (16, 1, 1)]


def layer_sizes():
    return [cout * ks * ks * cin for cin, cout, ks in LAYERS]


def num_params():
    return sum(layer_sizes())


def layer_offsets():
    off, out = 0, []
    for n in layer_sizes():
        out.append(off)
        off += n
    return out


def round_bf16(t):
    """float64 -> float32 -> bfloat16 (round to nearest even) -> float64."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _weights(w):
    """Flat weights -> list of conv2d kernels [cout, cin, ks, ks] (float64 tensors)."""
    w = torch.as_tensor(np.asarray(w, dtype=np.float64)) if not torch.is_tensor(w) else w
    out, off = [], 0
    for cin, cout, ks in LAYERS:
        n = cout * ks * ks * cin
        out.append(w[off:off + n].reshape(cout, ks, ks, cin).permute(0, 3, 1, 2))
        off += n
    return out


def _conv(x, k, relu, bf16):
    if bf16:
        x = x + (round_bf16(x) - x).detach()
        k = k + (round_bf16(k) - k).detach()
    y = F.conv2d(x, k, padding=k.shape[-1] // 2)
    return torch.relu(y) if relu else y


def _up(x):
    return x.repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)


def forward_t(w, x, bf16=False):
    """Network output [nb, H, W] for x [nb, H, W, 2] (torch float64, NHWC)."""
    k = _weights(w)
    h = x.permute(0, 3, 1, 2)
    a1 = _conv(h, k[0], True, bf16)
    s1 = _conv(a1, k[1], True, bf16)
    a2 = _conv(F.avg_pool2d(s1, 2), k[2], True, bf16)
    s2 = _conv(a2, k[3], True, bf16)
    a3 = _conv(F.avg_pool2d(s2, 2), k[4], True, bf16)
    b3 = _conv(a3, k[5], True, bf16)
    a4 = _conv(torch.cat([_up(b3), s2], dim=1), k[6], True, bf16)
    b4 = _conv(a4, k[7], True, bf16)
    a5 = _conv(torch.cat([_up(b4), s1], dim=1), k[8], True, bf16)
    b5 = _conv(a5, k[9], True, bf16)
    return _conv(b5, k[10], False, bf16)[:, 0]


def forward(w, x, bf16=False):
    with torch.no_grad():
        return forward_t(None if w is None else torch.as_tensor(np.asarray(w, np.float64)),
                         torch.as_tensor(np.asarray(x, np.float64)), bf16).numpy()


def loss_t(w, x, t, bf16=False):
    """Mean over the batch of ||y - t||^2 / ||t||^2."""
    y = forward_t(w, x, bf16)
    e = ((y - t) ** 2).sum(dim=(1, 2))
    n = (t ** 2).sum(dim=(1, 2))
    return (e / n).mean(), e / n


def loss_and_grad(w, x, t, bf16=False):
    """(mean loss, per-sample losses, gradient w.r.t. the flat weights) in float64."""
    wt = torch.tensor(np.asarray(w, np.float64), requires_grad=True)
    L, per = loss_t(wt, torch.as_tensor(np.asarray(x, np.float64)), torch.as_tensor(np.asarray(t, np.float64)), bf16)
    L.backward()
    return float(L), per.detach().numpy(), wt.grad.numpy().copy()


def loss(w, x, t, bf16=False):
    with torch.no_grad():
        L, per = loss_t(torch.as_tensor(np.asarray(w, np.float64)), torch.as_tensor(np.asarray(x, np.float64)),
                        torch.as_tensor(np.asarray(t, np.float64)), bf16)
    return float(L), per.numpy()


def adam_step(w, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1); step counts from 1.  Returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def net_input(r, H, alpha):
    """Sample [H, H, 2] from an n x n residual: r / rms(r) at the top-left n x n, 0 elsewhere; alpha channel.
    rms(r) = ||r|| / n, the root mean square over the n x n interior."""
    r = np.asarray(r, np.float64)
    n = r.shape[0]
    x = np.zeros((H, H, 2))
    rms = np.sqrt((r * r).sum()) / n
    x[:n, :n, 0] = r / rms if rms > 0 else r
    x[:, :, 1] = alpha
    return x


def apply(w, r, alpha, H, bf16=False):
    """Preconditioner action z = rms(r) * Net(r / rms(r), alpha) on the n x n interior."""
    r = np.asarray(r, np.float64)
    n = r.shape[0]
    rms = np.sqrt((r * r).sum()) / n
    y = forward(w, net_input(r, H, alpha)[None], bf16)[0]
    return (rms if rms > 0 else 1.0) * y[:n, :n]


def forward_fp32(w, x):
    """The same network evaluated in FP32 on the CPU (torch float32 ops, the FP32 weights and
    inputs as given): an independent FP32 evaluation whose distance from the FP64 forward
    shows what FP32 arithmetic alone costs on a given input."""
    with torch.no_grad():
        wt = torch.as_tensor(np.asarray(w, np.float32))
        xt = torch.as_tensor(np.asarray(x, np.float32))
        return forward_t(wt, xt).to(torch.float64).numpy()
