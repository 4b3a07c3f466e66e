"""FP64 oracle of the learned velocity surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate stands in for the fine-grid lookup of the fluid velocity at a
particle (the "locally interpolated values" of Sec. 1): from the bulk fields
around the particle it predicts the sub-bulk part of the velocity,

    u_pred = u_bulk + s * y,   y = MLP(standardised features),

where u_bulk is the trilinear interpolation of the restricted bulk velocity and
s the per-component scale of the residual u_fine - u_bulk on the training set.

Features (193): the 27 bulk cells around the containing cell (dz, dy, dx in
-1..1, dx fastest, indices clamped at the walls), each (eps, U_x, U_y, U_z, G_x,
G_y, G_z) with eps = 1 - phi; then the in-cell offsets x/h - i (three); then
d / h_x.  The 26 neighbour cells enter as differences from the centre cell (the
centre cell as its own values): an invertible linear re-encoding of the same
stencil that keeps the sub-bulk curvature, a percent of the field values,
above the BF16 rounding of the standardised inputs.  Each feature is
standardised with the training-set mean and standard deviation (floored, see
norm_stats).

Network: 193 -> 128 -> 128 -> 128 -> 3, tanh-form GELU after the three hidden
layers, linear output.  The GPU rounds to BF16 (round to nearest even) the
weights and the input of every product, and accumulates in FP32; this oracle
rounds at the same points and accumulates in FP64.  Rounding points:

  forward   X0 = bf16(x~);  Z_l = bf16(A_{l-1}) @ bf16(W_l) + b_l;  A_l = gelu(Z_l)
  loss      L = (1/B) sum_p 1/2 |y_p - t_p|^2,  dY = (Y - T) / B
  backward  dW_l = bf16(A_{l-1})^T @ bf16(dZ_l),  db_l = sum_p dZ_l
            dA_{l-1} = bf16(dZ_l) @ bf16(W_l)^T,  dZ_{l-1} = dA_{l-1} * gelu'(Z_{l-1})
  Adam      FP32 master weights, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected.

Weights are stored W_l[k][n] (fan-in rows), biases b_l[n].  The feature vector
is zero-padded to KIN = 208 (a multiple of 16) and the output to 3 values.
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 193
KIN = 208
HIDDEN = 128
NOUT = 3
LAYERS = [(NFEAT, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, NOUT)]
GELU_C = math.sqrt(2.0 / math.pi)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    The value is first rounded to binary32 (as the GPU holds it), then its
    16 low-order bits are rounded away."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out.reshape(np.shape(x))


def gelu(z):
    """0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))"""
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    """Derivative of the tanh-form GELU."""
    u = GELU_C * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    du = GELU_C * (1.0 + 3 * 0.044715 * z ** 2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def init_params(seed=0):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, FP32 values."""
    rng = np.random.default_rng(seed)
    params = []
    for fin, fout in LAYERS:
        b = math.sqrt(6.0 / fin)
        W = rng.uniform(-b, b, size=(fin, fout)).astype(np.float32).astype(np.float64)
        params.append((W, np.zeros(fout)))
    return params


# ---------------------------------------------------------------------------
# Features and targets
# ---------------------------------------------------------------------------

def features(pos, diam, eps_b, U, G, box, nb, prec32=True):
    """[n, 193] raw (unstandardised) features; bulk fields are flat [ncell] /
    [3, ncell] arrays in x-fastest order.  The containing cell is the binning's
    (the same clamp and index rule, decided in binary32 when ``prec32``); the
    offset is the clamped position over h minus that index."""
    from . import bin_particles
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    nb = [int(v) for v in nb]
    box = [float(v) for v in box]
    h = [box[a] / nb[a] for a in range(3)]
    if prec32:
        L32 = np.asarray(box, dtype=np.float32)
        x = np.minimum(np.maximum(pos.astype(np.float32), np.float32(0)), L32).astype(np.float64)
    else:
        x = np.minimum(np.maximum(pos, 0.0), np.asarray(box))
    x = np.where(np.isnan(x), 0.0, x)
    cell, _ = bin_particles(pos, box, nb, prec32)
    cell = cell.astype(np.int64)
    idx = np.stack([cell % nb[0], (cell // nb[0]) % nb[1], cell // (nb[0] * nb[1])], axis=1)
    fields = [np.asarray(eps_b, dtype=np.float64).ravel()] + \
             [np.asarray(U, dtype=np.float64).reshape(3, -1)[a] for a in range(3)] + \
             [np.asarray(G, dtype=np.float64).reshape(3, -1)[a] for a in range(3)]
    out = np.empty((n, NFEAT))
    col = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ci = np.clip(idx[:, 0] + dx, 0, nb[0] - 1)
                cj = np.clip(idx[:, 1] + dy, 0, nb[1] - 1)
                ck = np.clip(idx[:, 2] + dz, 0, nb[2] - 1)
                c = ci + nb[0] * (cj + nb[1] * ck)
                for f in fields:
                    out[:, col] = f[c] if (dx, dy, dz) == (0, 0, 0) else f[c] - f[cell]
                    col += 1
    for a in range(3):
        out[:, col] = x[:, a] / h[a] - idx[:, a]
        col += 1
    out[:, col] = np.asarray(diam, dtype=np.float64).ravel() / h[0]
    return out


def residual_target(u_fine, u_bulk):
    """The surrogate's target: the sub-bulk part of the fluid velocity at the
    particle, fine-grid lookup minus bulk trilinear interpolation."""
    return np.asarray(u_fine, dtype=np.float64) - np.asarray(u_bulk, dtype=np.float64)


def target_scale(R):
    """Per-component standard deviation of the residuals; a component with no
    spread (e.g. a field with no w) takes the largest of the others, or 1."""
    s = np.asarray(R, dtype=np.float64).reshape(-1, 3).std(axis=0)
    big = s.max()
    s[s < 1e-12 * max(big, 1e-300)] = big if big > 0 else 1.0
    if big == 0:
        s[:] = 1.0
    return s


def predict(params, X, mean, std, scale, u_bulk, emulate=True):
    """Fluid velocity at the particles: bulk interpolation plus the scaled
    network output."""
    Y, _ = forward(params, standardise(X, mean, std), emulate)
    return np.asarray(u_bulk, dtype=np.float64) + Y * np.asarray(scale, dtype=np.float64)


def standardise(X, mean, std):
    Xs = (np.asarray(X, dtype=np.float64) - mean) / std
    out = np.zeros((Xs.shape[0], KIN))
    out[:, :NFEAT] = Xs
    return out


STD_REL_FLOOR = 1e-4


def norm_stats(X):
    """Mean and population standard deviation per feature, with two floors.

    A neighbour-difference feature's std is raised to at least 1e-4 times the
    std of the centre cell's value of the same channel: a field that does not
    vary along some direction (such as a pressure gradient component across the
    flow) leaves differences that are pure FP32 rounding, which standardisation
    would otherwise blow up to O(1) inputs.  Then a feature with std below 1e-12
    gets std 1."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    centre = std[7 * 13:7 * 14].copy()
    for u in range(27):
        if u != 13:
            sl = slice(7 * u, 7 * u + 7)
            std[sl] = np.maximum(std[sl], STD_REL_FLOOR * centre)
    std[std < 1e-12] = 1.0
    return mean, std


# ---------------------------------------------------------------------------
# Forward, backward, Adam
# ---------------------------------------------------------------------------

def forward(params, Xs, emulate=True):
    """Returns (Y [n,3], cache).  ``Xs`` is standardised and padded [n, KIN]."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    A = r(Xs)[:, :NFEAT]
    cache = {"A": [A], "Z": []}
    for l, (W, b) in enumerate(params):
        Z = r(A) @ r(W) + b
        cache["Z"].append(Z)
        if l < len(params) - 1:
            A = gelu(Z)
            cache["A"].append(A)
        else:
            A = Z
    return A, cache


def loss_and_grads(params, Xs, T, emulate=True):
    """Mean-over-batch 1/2 |y - t|^2 and its gradients [(dW, db)] per layer."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    Y, cache = forward(params, Xs, emulate)
    B = Y.shape[0]
    D = Y - T
    loss = 0.5 * float((D * D).sum()) / B
    dZ = D / B
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        Aprev = cache["A"][l]
        grads[l] = (r(Aprev).T @ r(dZ), dZ.sum(axis=0))
        if l > 0:
            dA = r(dZ) @ r(W).T
            dZ = dA * gelu_grad(cache["Z"][l - 1])
    return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * g
                v = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                self.m[i] = tuple(m if k == j else self.m[i][k] for k in range(2))
                self.v[i] = tuple(v if k == j else self.v[i][k] for k in range(2))
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append(tuple(new))
        return out


def flatten(params):
    """FP32 flat parameter vector: W1, b1, W2, b2, ... (row-major W[k][n])."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflatten(vec):
    vec = np.asarray(vec, dtype=np.float64)
    params, o = [], 0
    for fin, fout in LAYERS:
        W = vec[o:o + fin * fout].reshape(fin, fout)
        o += fin * fout
        b = vec[o:o + fout]
        o += fout
        params.append((W, b))
    return params


NPARAM = sum(fin * fout + fout for fin, fout in LAYERS)
