"""O5: the learned surrogate of the path variables, FP64 reference.

Test infrastructure only (see ``oracle/__init__.py``).

The surrogate is not in the paper: it maps a structure, aligned onto a fixed
reference by the same optimal superposition as Eq. 3 (Section 3), to the path
variables (s, z) of Eq. 2 with a multilayer perceptron, and gets ds/dx and
dz/dx by differentiating the network and the alignment.

Network: input 3n aligned coordinates, hidden layers with SiLU
(v / (1 + e^-v)), a linear output of 2 standardised values
(s - mu_s) / sd_s and (z - mu_z) / sd_z.  Weights W_l are [fan_in][fan_out]
(pre = a @ W + b).

Rounding points (``rounded=True``): the HIP kernels multiply BF16 operands
with FP32 accumulation, so every GEMM operand (layer input, weight, backward
signal) is rounded to BF16 (round to nearest even, via FP32) before an exact
FP64 product here; biases, pre-activations, SiLU and the loss stay FP64.
``rounded=False`` gives the plain FP64 network the finite-difference pins
use.

Training: mean over the batch of the squared error summed over the two
outputs; Adam (Kingma and Ba) on FP64 master weights.

Parity unpinned: the accuracy the trained network reaches on a given walk.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .msd import centre, normalise_weights, rotation_adjoint, rotation_term, superpose

__all__ = ["bf16", "silu", "silu_grad", "MLP", "forward", "input_grad", "param_grads", "loss_and_grad",
           "adam_step", "align", "surrogate", "surrogate_fd_check_fn"]


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (8-bit mantissa), nearest even, through FP32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(v):
    v = np.asarray(v, dtype=np.float64)
    return v / (1.0 + np.exp(-v))


def silu_grad(v):
    """d/dv [v sigma(v)] = sigma(v) (1 + v (1 - sigma(v)))."""
    v = np.asarray(v, dtype=np.float64)
    sg = 1.0 / (1.0 + np.exp(-v))
    return sg * (1.0 + v * (1.0 - sg))


@dataclass
class MLP:
    """Weights [fan_in][fan_out] and biases per layer (FP64 masters)."""
    W: list
    b: list
    mean: np.ndarray = field(default_factory=lambda: np.zeros(2))   # mu_s, mu_z
    std: np.ndarray = field(default_factory=lambda: np.ones(2))     # sd_s, sd_z

    @property
    def sizes(self):
        return [self.W[0].shape[0]] + [w.shape[1] for w in self.W]


def _r(x, rounded):
    return bf16(x) if rounded else np.asarray(x, dtype=np.float64)


def forward(net: MLP, X, *, rounded: bool = True) -> dict:
    """Forward pass on a batch X [B][fan_in].  Returns the standardised
    output ``y`` [B][2] and the cache the backward pass needs."""
    a = np.asarray(X, dtype=np.float64)
    acts, pres = [], []
    L = len(net.W)
    for l in range(L):
        ar = _r(a, rounded)
        acts.append(ar)
        pre = ar @ _r(net.W[l], rounded) + net.b[l]
        pres.append(pre)
        a = silu(pre) if l < L - 1 else pre
    return {"y": a, "acts": acts, "pres": pres}


def _backward(net: MLP, cache: dict, dy, rounded: bool):
    """Signals d_l = dLoss/dpre_l for every layer, last layer first."""
    L = len(net.W)
    d = np.asarray(dy, dtype=np.float64)
    ds = [None] * L
    ds[L - 1] = d
    for l in range(L - 1, 0, -1):
        g = _r(d, rounded) @ _r(net.W[l], rounded).T
        d = g * silu_grad(cache["pres"][l - 1])
        ds[l - 1] = d
    return ds


def input_grad(net: MLP, cache: dict, dy, *, rounded: bool = True) -> np.ndarray:
    """d(dy . y)/dX [B][fan_in] (dy [B][2] weights the two outputs)."""
    ds = _backward(net, cache, dy, rounded)
    return _r(ds[0], rounded) @ _r(net.W[0], rounded).T


def param_grads(net: MLP, cache: dict, dy, *, rounded: bool = True):
    """(dW_l, db_l) of sum_b dy_b . y_b."""
    ds = _backward(net, cache, dy, rounded)
    dW = [cache["acts"][l].T @ _r(ds[l], rounded) for l in range(len(net.W))]
    db = [ds[l].sum(axis=0) for l in range(len(net.W))]
    return dW, db


def loss_and_grad(y, t):
    """Mean over the batch of sum_k (y_k - t_k)^2, and its gradient in y."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    r = y - t
    return float((r * r).sum() / B), 2.0 * r / B


def adam_step(w, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (bias-corrected moments); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def align(x, ref, w=None):
    """Superpose the reference onto x (Eq. 3 machinery) and express x in the
    reference frame: x' = R^T (x - c_x) with R mapping ref onto x.
    Returns (x' [n][3], the superposition record)."""
    x = np.asarray(x, dtype=np.float64)
    sp = superpose(x, ref, w, w)
    xp = sp.x_c @ sp.R        # row k: R^T x_c,k
    return xp, sp


def surrogate(net: MLP, x, ref, w=None, *, rounded: bool = True):
    """(s, z) of the surrogate for one structure x [n][3] and their
    gradients with respect to the raw coordinates [n][3] (alignment,
    rotation derivative and centring included)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    wn = normalise_weights(w, n)
    xp, sp = align(x, ref, wn)
    cache = forward(net, xp.reshape(1, -1), rounded=rounded)
    y = cache["y"][0]
    s = net.mean[0] + net.std[0] * y[0]
    z = net.mean[1] + net.std[1] * y[1]
    grads = []
    for k in range(2):
        dy = np.zeros((1, 2))
        dy[0, k] = net.std[k]
        g = input_grad(net, cache, dy, rounded=rounded).reshape(n, 3)   # df/dx'
        grads.append(_chain_alignment(g, sp, wn))
    return s, z, grads[0], grads[1]


def _chain_alignment(g, sp, wn):
    """d f(x'(x))/dx for x' = R(x)^T (x - c(x)), given g = df/dx'.

    * explicit part: R g_k, with the centring projection -w_k sum_j R g_j;
    * rotation part: f depends on R through x'_k[b] = sum_a R_ab x_c,k[a],
      so G_ab = sum_k x_c,k[a] g_k[b]; the top-eigenvector perturbation turns
      G into Gamma = d(G:R)/dM for M = sum_j w_j a_c,j x_c,j^T, whose
      derivative in x_k is w_k (Gamma^T a_c,k) (Section 3 machinery, the same
      adjoint as the close-structure derivative of Eq. 6).
    """
    R = sp.R
    explicit = g @ R.T                                  # row k: R g_k
    explicit = explicit - wn[:, None] * explicit.sum(axis=0)[None, :]
    G = sp.x_c.T @ g                                    # G_ab = sum_k x_c,k[a] g_k[b]
    Gamma = rotation_adjoint(sp.evals, sp.evecs, G)
    return explicit + rotation_term(Gamma, sp.a_c, wn)


def surrogate_fd_check_fn(net: MLP, ref, w=None):
    """f(x) -> (s, z) in FP64 without rounding (for finite differences)."""
    def f(x):
        s, z, _, _ = surrogate(net, x, ref, w, rounded=False)
        return np.array([s, z])
    return f
