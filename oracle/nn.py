"""FP64 NumPy reference of the warm-start network (test infrastructure only).

Same architecture and parameter layout as the GPU network (declared with the warm-start
API of the C header): three stride-2, width-5, pad-2 convolutions over 256 positions with
ReLU, two hidden fully connected layers with ReLU, a linear coefficient layer and the fixed
synthesis basis cos(q pi t) sin(p pi x / 2).  Loss: mean over the batch of
||U - T/r||^2 / ||T/r||^2.  Backward is written out by the chain rule; it is pinned by
central finite differences in the tests.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class NetConfig:
    m: int
    s: int
    conv_ch: tuple = (96, 96, 64)
    fc: tuple = (768, 512)
    nx: int = 32
    nt: int = 16

    @property
    def cin(self) -> int:
        return self.s + 4

    def layer_shapes(self):
        """[(kin, kout, is_conv, relu, lin, lout, cin)] in parameter order."""
        ch = (self.cin,) + tuple(self.conv_ch)
        pos = (256, 128, 64, 32)
        out = [(5 * ch[i], ch[i + 1], True, True, pos[i], pos[i + 1], ch[i]) for i in range(3)]
        fin = (32 * ch[3], self.fc[0], self.fc[1])
        fout = (self.fc[0], self.fc[1], self.nx * self.nt)
        out += [(fin[i], fout[i], False, i < 2, 1, 1, 0) for i in range(3)]
        return out

    def num_params(self) -> int:
        return sum(k * n + n for k, n, *_ in self.layer_shapes())


def unpack(cfg: NetConfig, theta: np.ndarray):
    """Split the flat parameter vector into [(W [kin][kout], b [kout])]."""
    res, off = [], 0
    for kin, kout, *_ in cfg.layer_shapes():
        W = theta[off:off + kin * kout].reshape(kin, kout)
        off += kin * kout
        b = theta[off:off + kout]
        off += kout
        res.append((W, b))
    return res


def synthesis_basis(cfg: NetConfig) -> np.ndarray:
    """Bsyn [nx*nt][s*m]: row q*nx + p is cos(q pi t_{n+1}) sin((p+1) pi x_i / 2) sqrt(2/(s m))."""
    t = np.arange(1, cfg.s + 1) / cfg.s
    x = 2.0 * np.arange(1, cfg.m + 1) / (cfg.m + 1)
    rows = []
    for q in range(cfg.nt):
        for p in range(cfg.nx):
            rows.append(np.outer(np.cos(q * np.pi * t), np.sin((p + 1) * np.pi * x / 2.0)).reshape(-1))
    return np.array(rows) * np.sqrt(2.0 / (cfg.s * cfg.m))


def features(cfg: NetConfig, f: np.ndarray, d_plus: np.ndarray, d_minus: np.ndarray, alpha: float):
    """X [256][cin]: channel c <= s is f[c]/r (r = RMS of f), then d+, d-, alpha - 1.5; rows
    i >= m are zero.  Returns (X, r)."""
    r = np.sqrt(np.mean(f ** 2))
    if not r > 0:
        r = 1.0
    X = np.zeros((256, cfg.cin))
    X[:cfg.m, :cfg.s + 1] = (f / r).T
    X[:cfg.m, cfg.s + 1] = d_plus
    X[:cfg.m, cfg.s + 2] = d_minus
    X[:cfg.m, cfg.s + 3] = alpha - 1.5
    return X, r


def _id(x):
    return x


def conv_forward(X: np.ndarray, W: np.ndarray, b: np.ndarray, lout: int, q=_id) -> np.ndarray:
    """out[o][co] = b[co] + sum_{t<5} sum_c X[2o + t - 2][c] W[t*C + c][co] (X zero outside).
    q rounds the operands of every product (identity: exact FP64)."""
    X, W = q(X), q(W)
    L, C = X.shape
    out = np.tile(b, (lout, 1)).astype(np.float64)
    for t in range(5):
        src = 2 * np.arange(lout) + t - 2
        ok = (src >= 0) & (src < L)
        out[ok] += X[src[ok]] @ W[t * C:(t + 1) * C]
    return out


def conv_backward(X: np.ndarray, W: np.ndarray, dOut: np.ndarray, q=_id):
    """Gradients of conv_forward w.r.t. W, b and X (q as in conv_forward; the bias gradient
    sums the unrounded dOut)."""
    db = dOut.sum(axis=0)
    X, W, dOut = q(X), q(W), q(dOut)
    L, C = X.shape
    lout = dOut.shape[0]
    dW = np.zeros_like(W)
    dX = np.zeros_like(X)
    for t in range(5):
        src = 2 * np.arange(lout) + t - 2
        ok = (src >= 0) & (src < L)
        dW[t * C:(t + 1) * C] += X[src[ok]].T @ dOut[ok]
        np.add.at(dX, src[ok], dOut[ok] @ W[t * C:(t + 1) * C].T)
    return dW, db, dX


def forward(cfg: NetConfig, theta: np.ndarray, X: np.ndarray, q=_id):
    """U [s*m] for one instance's features X; also returns the cached activations.  q rounds
    the operands of every matrix product (identity: exact FP64; a bf16 rounding reproduces a
    network that multiplies bf16 operands)."""
    params = unpack(cfg, theta)
    shapes = cfg.layer_shapes()
    acts = [X]
    h = X
    for (W, b), (kin, kout, conv, relu, lin, lout, cin) in zip(params, shapes):
        if conv:
            z = conv_forward(h, W, b, lout, q)
        else:
            z = q(h.reshape(-1)) @ q(W) + b
        h = np.maximum(z, 0.0) if relu else z
        acts.append(h)
    U = q(acts[-1]) @ q(synthesis_basis(cfg))
    return U, acts


def loss_and_grad(cfg: NetConfig, theta: np.ndarray, Xs, Ts, rs, q=_id):
    """Mean relative MSE over the batch and its gradient w.r.t. theta (q as in forward)."""
    B = len(Xs)
    Bsyn = synthesis_basis(cfg)
    params = unpack(cfg, theta)
    shapes = cfg.layer_shapes()
    grad = np.zeros_like(theta)
    gparts = unpack(cfg, grad)  # views into grad
    total = 0.0
    for X, T, r in zip(Xs, Ts, rs):
        U, acts = forward(cfg, theta, X, q)
        tv = T / r
        den = float(tv @ tv)
        total += float((U - tv) @ (U - tv)) / den
        dU = 2.0 * (U - tv) / (den * B)
        d = q(Bsyn) @ q(dU)
        for li in range(5, -1, -1):
            W, b = params[li]
            kin, kout, conv, relu, lin, lout, cin = shapes[li]
            out = acts[li + 1]
            if relu:
                d = d * (out > 0)
            hin = acts[li]
            gW, gb = gparts[li]
            if conv:
                dW, db, dX = conv_backward(hin, W, d, q)
                gW += dW
                gb += db
                d = dX
            else:
                gW += np.outer(q(hin.reshape(-1)), q(d))
                gb += d
                d = (q(W) @ q(d)).reshape(hin.shape)
    return total / B, grad
