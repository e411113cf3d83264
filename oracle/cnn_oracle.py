"""CPU oracle of the decode-time predictor used for learned scheduling.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain PyTorch CPU
ops in float64.  The predictor is not part of the paper: it is a small
convolutional network that estimates ln(1 + T_dec) of a noise sample from
its syndrome, where T_dec is the decoding time of Sec. 5.1 (Def. "logical
failure rate, expected decoding time, and thresholds").  It only orders and
groups work; decoding results never depend on it.

Network (parameters as one float32 vector of CNN_PARAMS = 7137 values):
  input   x[y][x] = (number of anyons in the B x B block (y, x)) / 8,
          an M x M map, M = L / B
  layer 1 conv 3x3, 1 -> 16 channels, circular padding, bias, ReLU
  layer 2..4 conv 3x3, 16 -> 16, circular padding, bias, ReLU
  pool    global max over positions, per channel (first position in
          row-major order on ties)
  head    pred = bl + sum_c Wl[c] * feat[c]
Convolutions are cross-correlations:
  z[co][y][x] = b[co] + sum_{dy,dx in -1..1} sum_ci W[co][tap][ci] a[ci][(y+dy)%M][(x+dx)%M]
with tap = 3 (dy + 1) + (dx + 1).

Precision modes: "f64" computes everything in float64 (for finite-difference
checks); "bf16" rounds to bfloat16 (round to nearest even, via float32) at
the points where the GPU stores bfloat16: conv weights of layers 1-4, and the
activations of layers 1-3.  Layer-4 activations, biases and the head stay
in float32 precision or wider.  Rounding is treated as the identity in the
backward pass, so gradients are those of the float weights.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

C = 16
CNN_PARAMS = 7137
# offsets into the parameter vector
OFF_W1, OFF_B1 = 0, 144            # W1 [16 co][9 tap]
OFF_W2, OFF_B2 = 160, 2464         # W2 [16 co][9 tap][16 ci]
OFF_W3, OFF_B3 = 2480, 4784
OFF_W4, OFF_B4 = 4800, 7104
OFF_WL, OFF_BL = 7120, 7136        # head [16], bias [1]
CONV = ((OFF_W1, OFF_B1, 1), (OFF_W2, OFF_B2, C), (OFF_W3, OFF_B3, C), (OFF_W4, OFF_B4, C))
INIT_TAG = 0x636E6E31  # second counter word of the initializer's generator


def round_bf16(t: torch.Tensor) -> torch.Tensor:
    """Value of t rounded to float32, then to bfloat16 (nearest, ties to even)."""
    return t.float().bfloat16().double()


def _ste(t: torch.Tensor) -> torch.Tensor:
    return t + (round_bf16(t.detach()) - t.detach())


def _conv_weight(params: torch.Tensor, off: int, cin: int) -> torch.Tensor:
    # [co][tap][ci] -> torch's [co][ci][ky][kx]
    w = params[off:off + C * 9 * cin].reshape(C, 9, cin)
    return w.permute(0, 2, 1).reshape(C, cin, 3, 3)


def block_counts(sigma: np.ndarray, B: int = 8) -> np.ndarray:
    """Anyons per B x B block of a [.., L, L] 0/1 syndrome map, as uint8 [.., L/B, L/B]."""
    s = np.asarray(sigma, dtype=np.int64)
    L = s.shape[-1]
    M = L // B
    c = s.reshape(s.shape[:-2] + (M, B, M, B)).sum(axis=(-3, -1))
    return c.astype(np.uint8)


def forward(counts, params, mode: str = "bf16", requires_grad: bool = False):
    """Forward pass.  counts: uint8 [n, M, M]; params: float [7137].

    Returns a dict with pred [n] (float64 tensor), feat [n, 16], argmax
    [n, 16] (row-major position of the maximum, numpy int64), the stored
    activations a1..a3 and a4 and the float64 parameter tensor (with
    gradient tracking if requested)."""
    if mode not in ("bf16", "f64"):
        raise ValueError(mode)
    p = torch.as_tensor(np.asarray(params, dtype=np.float32)).double()
    if mode == "f64":
        p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    p = p.clone().requires_grad_(requires_grad)
    x = torch.as_tensor(np.asarray(counts, dtype=np.float64)).unsqueeze(1) / 8.0
    n, M = x.shape[0], x.shape[-1]
    a = x
    acts = []
    for layer, (ow, ob, cin) in enumerate(CONV):
        w = _conv_weight(p, ow, cin)
        if mode == "bf16":
            w = _ste(w)
        z = F.conv2d(F.pad(a, (1, 1, 1, 1), mode="circular"), w) + p[ob:ob + C].reshape(1, C, 1, 1)
        if mode == "bf16":  # the GPU accumulates in float32
            z = z + (z.detach().float().double() - z.detach())
        a = torch.relu(z)
        if mode == "bf16" and layer < 3:
            a = _ste(a)
        acts.append(a)
    flat = acts[3].reshape(n, C, M * M)
    idx = np.argmax(flat.detach().numpy(), axis=2)  # first maximum
    feat = torch.gather(flat, 2, torch.as_tensor(idx).unsqueeze(2)).squeeze(2)
    pred = feat @ p[OFF_WL:OFF_WL + C] + p[OFF_BL]
    return {"pred": pred, "feat": feat, "argmax": idx, "acts": acts, "params": p}


def loss_and_grad(counts, params, target, mode: str = "bf16"):
    """Mean squared error of pred against target (ln(1 + T_dec)) over the
    batch and its gradient with respect to the parameters (float64 [7137])."""
    out = forward(counts, params, mode, requires_grad=True)
    y = torch.as_tensor(np.asarray(target, dtype=np.float64))
    loss = ((out["pred"] - y) ** 2).mean()
    loss.backward()
    return float(loss.detach()), out["params"].grad.numpy().copy(), out


def init_params(seed: int, philox) -> np.ndarray:
    """Initial parameters: conv and head weights uniform in +-sqrt(6 / fan_in)
    (He et al., 2015, uniform form), biases zero.  Parameter j draws word 0
    of Philox4x32-10 at counter (j, INIT_TAG, 0, 0) under key (seed lo, seed
    hi): u = (word + 1/2) / 2^32, w = (2u - 1) * bound, in float64, then
    float32."""
    out = np.zeros(CNN_PARAMS, dtype=np.float32)
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    for off, count, fan in ((OFF_W1, 144, 9), (OFF_W2, 2304, 144), (OFF_W3, 2304, 144),
                            (OFF_W4, 2304, 144), (OFF_WL, 16, 16)):
        bound = float(np.sqrt(6.0 / fan))
        for j in range(off, off + count):
            w0 = int(philox([j, INIT_TAG, 0, 0], key)[0])
            u = (w0 + 0.5) / 4294967296.0
            out[j] = np.float32((2.0 * u - 1.0) * bound)
    return out


def init_bound(j: int) -> float:
    """sqrt(6 / fan_in) of parameter j (0 for biases)."""
    for off, count, fan in ((OFF_W1, 144, 9), (OFF_W2, 2304, 144), (OFF_W3, 2304, 144),
                            (OFF_W4, 2304, 144), (OFF_WL, 16, 16)):
        if off <= j < off + count:
            return float(np.sqrt(6.0 / fan))
    return 0.0


def adam_step(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1) in float64.  step is
    the 1-based update count.  Returns new (params, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
