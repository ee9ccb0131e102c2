"""FP64 reference of the learned per-mode preconditioner.  TEST INFRASTRUCTURE ONLY.

Network 514 -> 256 -> 256 -> 512 with ReLU hidden layers, loss
(1/2n) sum_i |y_i - t_i|^2, parameters in the order W1 [256][514], b1, W2
[256][256], b2, W3 [512][256], b3.  ``forward``/``gradients`` follow the
definition in FP64.  With ``bf16=True`` they round, at the same points as the
matrix-core path, the quantities that path stores in BF16 (weights, inputs,
hidden activations, and in the backward pass dY and the masked dZ) and keep
everything else in FP64, so that the GPU result differs from it only by FP32
accumulation order.

Mode transforms (the preconditioner's input and output):
  R_m[node] = (1/2M) sum_j r[node, j] e^{-i m theta_j},  m = -M+1..M,
  x_m = [Re R_m / s_m, Im R_m / s_m, k/30, m/M],  s_m = |R_m|_2,
  e[node, j] = sum_m s_m (y_m[:256] + i y_m[256:]) e^{i m theta_j}.
"""
import numpy as np

N_IN, N_H, N_OUT = 514, 256, 512
SHAPES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_OUT, N_H), (N_OUT,)]


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32).view(np.float32)).astype(np.float64)


def split(params):
    out, o = [], 0
    for sh in SHAPES:
        n = int(np.prod(sh))
        out.append(np.asarray(params[o:o + n], dtype=np.float64).reshape(sh))
        o += n
    return out


def param_count():
    return sum(int(np.prod(sh)) for sh in SHAPES)


def forward(params, x, bf16=False):
    W1, b1, W2, b2, W3, b3 = split(params)
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    if bf16:
        W1, W2, W3 = rnd(W1), rnd(W2), rnd(W3)
    x = rnd(x)
    z1 = x @ W1.T + b1
    a1 = rnd(np.maximum(z1, 0.0))
    z2 = a1 @ W2.T + b2
    a2 = rnd(np.maximum(z2, 0.0))
    y = a2 @ W3.T + b3
    return y, (x, a1, a2, W1, W2, W3)


def gradients(params, x, t, bf16=False):
    """(loss, gradient vector) of (1/2n) sum |y - t|^2."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    y, (xr, a1, a2, W1, W2, W3) = forward(params, x, bf16)
    n = x.shape[0]
    d = y - t
    loss = 0.5 * np.sum(d * d) / n
    dy = rnd(d / n)
    gW3 = dy.T @ a2
    gb3 = dy.sum(0)
    dz2 = rnd((dy @ W3) * (a2 > 0))
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(0)
    dz1 = rnd((dz2 @ W2) * (a1 > 0))
    gW1 = dz1.T @ xr
    gb1 = dz1.sum(0)
    return loss, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def modes(r, M, nodes):
    """R[m + M - 1, node] from r [nodes * 2M] (node-major)."""
    r = np.asarray(r).reshape(nodes, 2 * M)
    th = np.pi * np.arange(2 * M) / M
    ms = np.arange(-M + 1, M + 1)
    E = np.exp(-1j * np.outer(th, ms)) / (2 * M)          # [j, m]
    return (r @ E).T                                     # [m, node]


def features(r, M, nodes, k):
    R = modes(r, M, nodes)
    s = np.linalg.norm(R, axis=1)
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    ms = np.arange(-M + 1, M + 1)
    x = np.concatenate([R.real * inv[:, None], R.imag * inv[:, None],
                        np.full((2 * M, 1), k / 30.0), (ms / M)[:, None]], axis=1)
    return x, s


def targets(e, scale, M, nodes):
    E = modes(e, M, nodes)
    inv = np.where(scale > 0, 1.0 / np.where(scale > 0, scale, 1.0), 0.0)
    return np.concatenate([E.real * inv[:, None], E.imag * inv[:, None]], axis=1)


def reconstruct(y, scale, M, nodes):
    E = scale[:, None] * (y[:, :nodes] + 1j * y[:, nodes:])     # [m, node]
    th = np.pi * np.arange(2 * M) / M
    ms = np.arange(-M + 1, M + 1)
    return (E.T @ np.exp(1j * np.outer(ms, th))).reshape(-1)    # [node, j]


def precondition(params, v, M, nodes, k, bf16=True):
    x, s = features(v, M, nodes, k)
    y, _ = forward(params, x, bf16)
    return reconstruct(y, s, M, nodes)
