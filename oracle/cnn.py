"""Oracle of the learned peak filter (test infrastructure: only tests,
smoke() and bench.py's cpu_baseline leg use it).

The paper asks for efficiency and purity improvements of the peak finding
(section "Summary"); the filter scores each threshold peak from the
5 x 5 x 5 block of votes around it and drops low scores before refinement.
This module writes the network and its training step out plainly, in
float64, on the precision contract of the device kernels:

  * input: the votes of the window around the peak cell (phi0 periodic,
    q/pT and d0 outside the grid read 0), times 1/16 (exact in bfloat16 for
    votes below 4096);
  * every layer multiplies bfloat16-rounded inputs by bfloat16-rounded
    weights and accumulates wide (float32 on the device, float64 here); the
    bias is added after the sum; ReLU; the activation is rounded to bfloat16
    before it feeds the next layer;
  * network: conv3d 1->16 (3x3x3, valid) -> ReLU -> conv3d 16->16 (3x3x3,
    valid) -> ReLU -> linear 16->64 -> ReLU -> linear 64->1, a logit;
  * loss: binary cross-entropy with logits, positives weighted by pos_weight,
    mean over the batch; gradients of the float32 master weights through the
    same rounded activations (rounding treated as identity); the backward
    signals of the three hidden layers (dh3, dh2, dh1, after their ReLU
    masks) are rounded to bfloat16 like the activations before they enter
    the next contraction, which accumulates wide (the matrix-core training
    kernels take bfloat16 operands); dz and the last layer's gradients stay
    wide; SGD with momentum.

Flat parameter vector (float32 masters), in this order:
  W1[16][27] b1[16] W2[16][16][27] b2[16] W3[64][16] b3[64] W4[64] b4[1]
with tap t = (dk * 3 + dj) * 3 + di of a 3 x 3 x 3 kernel.
"""
from __future__ import annotations

import numpy as np

SHAPES = [("W1", (16, 27)), ("b1", (16,)), ("W2", (16, 16, 27)), ("b2", (16,)),
          ("W3", (64, 16)), ("b3", (64,)), ("W4", (64,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 8529
SCALE = 1.0 / 16.0


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def windows(acc, lins):
    """[N, 5, 5, 5] inputs (votes * 1/16) around the cells lins of the
    accumulator acc [n_d0][n_qpt][n_phi]: index order (dk, dj, di), each -2..2."""
    nd, nq, nphi = acc.shape
    lins = np.asarray(lins, np.int64)
    out = np.zeros((lins.size, 5, 5, 5), np.float64)
    for n, lin in enumerate(lins):
        i = lin % nphi
        col = lin // nphi
        j, k = col % nq, col // nq
        for a, dk in enumerate(range(-2, 3)):
            kk = k + dk
            if kk < 0 or kk >= nd:
                continue
            for b, dj in enumerate(range(-2, 3)):
                jj = j + dj
                if jj < 0 or jj >= nq:
                    continue
                for c, di in enumerate(range(-2, 3)):
                    out[n, a, b, c] = acc[kk, jj, (i + di) % nphi] * SCALE
    return out


def _patches(x):
    """3x3x3 patches of a [N, 5, 5, 5] (or [N, 5, 5, 5, C]) block: output
    position p = (a, b, c) in 0..2, tap t = (dk, dj, di)."""
    n = x.shape[0]
    tail = x.shape[4:]
    out = np.zeros((n, 27, 27) + tail, np.float64)
    for p in range(27):
        a, b, c = p // 9, (p // 3) % 3, p % 3
        for t in range(27):
            dk, dj, di = t // 9, (t // 3) % 3, t % 3
            out[:, p, t] = x[:, a + dk, b + dj, c + di]
    return out


def forward(flat, x, rounding=True):
    """Logits z [N] and the intermediate values (for backward).  rounding=False
    drops the bfloat16 roundings (the plain float64 network, for checks)."""
    rnd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    P = {k: rnd(v) if k[0] == "W" else v for k, v in unpack(flat).items()}
    x = rnd(x)
    X1 = _patches(x)                                     # [N, 27 pos, 27 taps]
    a1 = np.einsum("npt,ct->npc", X1, P["W1"]) + P["b1"]  # [N, 27, 16]
    h1 = rnd(np.maximum(a1, 0.0))
    a2 = np.einsum("npc,dcp->nd", h1, P["W2"]) + P["b2"]  # conv2 at its single output position
    h2 = rnd(np.maximum(a2, 0.0))
    a3 = h2 @ P["W3"].T + P["b3"]
    h3 = rnd(np.maximum(a3, 0.0))
    z = h3 @ P["W4"] + P["b4"][0]
    return z, dict(P=P, X1=X1, a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, h3=h3)


def loss_and_grad(flat, x, y, pos_weight=1.0, rounding=True):
    """Mean weighted BCE-with-logits and the gradient of the flat masters."""
    z, c = forward(flat, x, rounding)
    y = np.asarray(y, np.float64)
    w = np.where(y > 0.5, pos_weight, 1.0)
    sp = np.logaddexp(0.0, z)                       # softplus(z)
    loss = float(np.mean(w * (sp - y * z)))
    n = z.size
    dz = w * (1.0 / (1.0 + np.exp(-z)) - y) / n     # dL/dz
    P = c["P"]
    g = {}
    g["W4"] = dz @ c["h3"]
    g["b4"] = np.array([dz.sum()])
    rnd = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    dh3 = rnd(np.outer(dz, P["W4"]) * (c["a3"] > 0))
    g["W3"] = dh3.T @ c["h2"]
    g["b3"] = dh3.sum(0)
    dh2 = rnd((dh3 @ P["W3"]) * (c["a2"] > 0))
    g["W2"] = np.einsum("nd,npc->dcp", dh2, c["h1"])
    g["b2"] = dh2.sum(0)
    dh1 = rnd(np.einsum("nd,dcp->npc", dh2, P["W2"]) * (c["a1"] > 0))
    g["W1"] = np.einsum("npc,npt->ct", dh1, c["X1"])
    g["b1"] = dh1.sum((0, 1))
    return loss, pack(g), z


def sgd_step(flat, mom, grad, lr, momentum=0.9):
    """mom <- momentum * mom + grad; flat <- flat - lr * mom (float32 masters)."""
    mom = momentum * np.asarray(mom, np.float64) + grad
    new = np.asarray(flat, np.float64) - lr * mom
    return new.astype(np.float32), mom.astype(np.float32)


def init_params(seed):
    """He-style initial weights (float32), zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in SHAPES:
        if name[0] == "b":
            d[name] = np.zeros(shp)
        else:
            fan_in = {"W1": 27, "W2": 432, "W3": 16, "W4": 64}[name]
            d[name] = rng.normal(0.0, np.sqrt(2.0 / fan_in), shp)
    return pack(d).astype(np.float32)
