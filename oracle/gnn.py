"""Oracle: the learned initial-guess network, forward and analytic backward in fp64.

The network maps per-node features of the current right-hand side and the two
previous solutions to a correction of the extrapolated guess 2 phi^{n-1} - phi^{n-2}:

  features  X = [b/s_b, p1/s_p, p2/s_p, r_e/s_r, K d/s_r, d/s_d, dirichlet, 1]
            with e = 2 p1 - p2, d = p1 - p2, r_e = b - K e and s_* root-mean-square
            scales over all nodes (1 when zero)
  encoder   h0 = relu(X W0 + c0)                                  (8 -> 64)
  layers    m = mean over mesh neighbours (self excluded) of h
            h <- relu([h, m] W_l + c_l) + h,  l = 1, 2, 3          (128 -> 64)
  decoder   y = h w_d + c_d                                        (64 -> 1)
  guess     phi0 = (e + s_d y) on free nodes, 0 on Dirichlet nodes, then SMOOTH_SWEEPS
            damped Jacobi sweeps phi0 <- phi0 + (2/3) D^-1 (b - K phi0), which remove the
            high-frequency part of the network's error (cheap for a smoother, costly for
            a residual-based stopping rule) while keeping the smooth part it predicts

Training minimises the energy norm of the guess error measured in the scaled
output: L = (delta^T K delta) / N_free with delta = (y - y*) on free nodes and
y* = (phi* - e) / s_d, because the energy norm is what CG reduces.

``emulate=True`` rounds, as the device does, to bfloat16 (round to nearest
even): the weights of every matrix product, forward and backward, and in the
backward pass the other operands of the gradient products (layer inputs,
features and activation gradients).  Forward activations, features and the
neighbour mean are not rounded: the device carries them in fp32 and feeds the
matrix cores their bfloat16 high and low parts, which represent them to about
2^-17.  Biases, the decoder and all accumulations stay in high precision.
``emulate=False`` is plain fp64 (used for the finite-difference pin of the
backward pass).

Parameter vector (float32 on the device, float64 here), in this order:
W0 [16 x 64] (rows 8..15 multiply zero padding), c0 [64], then for l = 1..3
W_l [128 x 64] and c_l [64], then w_d [64] and c_d [1].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

HIDDEN = 64
SMOOTH_SWEEPS = 4
SMOOTH_OMEGA = 2.0 / 3.0
F_IN = 8
F_PAD = 16
LAYERS = 3


def param_shapes():
    shapes = [("W0", (F_PAD, HIDDEN)), ("c0", (HIDDEN,))]
    for l in range(1, LAYERS + 1):
        shapes += [(f"W{l}", (2 * HIDDEN, HIDDEN)), (f"c{l}", (HIDDEN,))]
    shapes += [("wd", (HIDDEN,)), ("cd", (1,))]
    return shapes


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in param_shapes():
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in param_shapes()])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def triangle_adjacency(n_nodes: int, tri: np.ndarray) -> sp.csr_matrix:
    """Node graph of the mesh: i ~ j when i and j are vertices of a common triangle."""
    t = np.asarray(tri, dtype=np.int64)
    rows = np.concatenate([t[:, a] for a in (0, 1, 2) for _ in (0, 1, 2)])
    cols = np.concatenate([t[:, b] for _ in (0, 1, 2) for b in (0, 1, 2)])
    a = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n_nodes, n_nodes))
    a.data[:] = 1.0
    return a


def neighbour_mean_operator(adjacency: sp.csr_matrix) -> sp.csr_matrix:
    """Row-normalised adjacency without the diagonal: (M h)_i = mean_{j ~ i, j != i} h_j."""
    a = sp.csr_matrix(adjacency, dtype=np.float64, copy=True)
    a.setdiag(0.0)
    a.eliminate_zeros()
    a.data[:] = 1.0
    deg = np.asarray(a.sum(axis=1)).ravel()
    deg[deg == 0] = 1.0
    return sp.diags(1.0 / deg) @ a


def _rms(a):
    r = float(np.sqrt(np.mean(a * a)))
    return r if r > 0 else 1.0


def features(k: sp.csr_matrix, dirichlet, b, p1, p2):
    """Returns (X [n x 8], e, s_d)."""
    e = 2.0 * p1 - p2
    d = p1 - p2
    re = b - k @ e
    kd = k @ d
    sb, sp_, sr, sd = _rms(b), _rms(p1), _rms(re), _rms(d)
    x = np.stack([b / sb, p1 / sp_, p2 / sp_, re / sr, kd / sr, d / sd,
                  np.asarray(dirichlet, dtype=np.float64), np.ones_like(b)], axis=1)
    return x, e, sd


def forward(theta, x, mean_op, emulate: bool = True):
    """Network output y and the saved intermediates."""
    p = unpack(theta)
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    xq = np.asarray(x, dtype=np.float64)
    a0 = xq @ r(p["W0"][:F_IN]) + p["c0"]
    h = np.maximum(a0, 0.0)
    cache = {"xq": xq, "a": [a0], "h": [h], "z": []}
    for l in range(1, LAYERS + 1):
        m = mean_op @ h
        z = np.concatenate([h, m], axis=1)
        a = z @ r(p[f"W{l}"]) + p[f"c{l}"]
        h = np.maximum(a, 0.0) + h
        cache["z"].append(z)
        cache["a"].append(a)
        cache["h"].append(h)
    y = h @ p["wd"] + p["cd"][0]
    return y, cache


def smooth(k: sp.csr_matrix, b, x, sweeps: int = SMOOTH_SWEEPS, omega: float = SMOOTH_OMEGA):
    """Damped Jacobi sweeps x <- x + omega D^-1 (b - K x), D = diag(K)."""
    dinv = 1.0 / k.diagonal()
    x = np.array(x, dtype=np.float64, copy=True)
    for _ in range(sweeps):
        x = x + omega * dinv * (b - k @ x)
    return x


def guess(theta, k, dirichlet, b, p1, p2, mean_op, emulate=True, sweeps: int = SMOOTH_SWEEPS):
    x, e, sd = features(k, dirichlet, b, p1, p2)
    y, _ = forward(theta, x, mean_op, emulate)
    free = 1.0 - np.asarray(dirichlet, dtype=np.float64)
    return smooth(k, b, (e + sd * y) * free, sweeps)


def loss_and_grad(theta, k, dirichlet, b, p1, p2, target, mean_op, emulate=True):
    """Energy-norm loss of the scaled output and its gradient w.r.t. theta."""
    p = unpack(theta)
    r = bf16 if emulate else (lambda v: np.asarray(v, dtype=np.float64))
    x, e, sd = features(k, dirichlet, b, p1, p2)
    y, c = forward(theta, x, mean_op, emulate)
    free = 1.0 - np.asarray(dirichlet, dtype=np.float64)
    nfree = max(float(free.sum()), 1.0)
    ystar = (target - e) / sd
    delta = (y - ystar) * free
    kdelta = k @ delta
    loss = float(delta @ kdelta) / nfree
    dy = 2.0 * kdelta * free / nfree                     # K symmetric
    g = {name: np.zeros(shape) for name, shape in param_shapes()}
    h3 = c["h"][-1]
    g["wd"] = h3.T @ dy
    g["cd"] = np.array([dy.sum()])
    dh = np.outer(dy, p["wd"])
    for l in range(LAYERS, 0, -1):
        a = c["a"][l]
        da = dh * (a > 0.0)
        daq = r(da)
        g[f"W{l}"] = r(c["z"][l - 1]).T @ daq
        g[f"c{l}"] = da.sum(axis=0)
        dz = daq @ r(p[f"W{l}"]).T
        dh = dh + dz[:, :HIDDEN] + mean_op.T @ dz[:, HIDDEN:]
    da0 = dh * (c["a"][0] > 0.0)
    da0q = r(da0)
    g["W0"][:F_IN] = r(c["xq"]).T @ da0q
    g["c0"] = da0.sum(axis=0)
    return loss, pack(g)
