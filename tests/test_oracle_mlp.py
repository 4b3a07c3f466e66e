"""Pins of the learned-surrogate oracle (oracle/mlp.py) against things it does not
compute itself: torch's own BF16 conversion and tanh-GELU, central finite
differences, hand-computed Adam steps, closed forms of the features for affine
and constant bulk fields, the zero residual of an affine fine field, and the
measured error of plain bulk interpolation on the Taylor-Green workloads."""
import math

import numpy as np
import pytest

import workload as W
from oracle import mlp as M


def test_param_count():
    # 193*128+128 + 2*(128*128+128) + 128*3+3
    assert M.NPARAM == 58243
    p = M.init_params(0)
    v = M.flatten(p)
    assert v.dtype == np.float32 and v.size == M.NPARAM
    q = M.unflatten(v)
    for (W1, b1), (W2, b2) in zip(p, q):
        np.testing.assert_array_equal(W1, W2)
        np.testing.assert_array_equal(b1, b2)


def test_bf16_matches_torch_and_ties():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, 65504.0, 1e-40, -3.3e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)
    # ties go to the even mantissa: ulp(1) in bfloat16 is 2^-7
    assert M.bf16(1 + 2.0 ** -8) == 1.0
    assert M.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6
    assert M.bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7


def test_gelu_closed_form_and_derivative():
    import torch
    z = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="tanh").numpy()
    np.testing.assert_allclose(M.gelu(z), ref, rtol=1e-14, atol=1e-15)
    assert M.gelu(0.0) == 0.0
    # the odd part of GELU is z/2: gelu(z) - gelu(-z) = z
    np.testing.assert_allclose(M.gelu(z) - M.gelu(-z), z, rtol=1e-13, atol=1e-13)
    hstep = 1e-5
    fd = (M.gelu(z + hstep) - M.gelu(z - hstep)) / (2 * hstep)
    np.testing.assert_allclose(M.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)
    assert abs(M.gelu_grad(0.0) - 0.5) < 1e-15


def _small_problem(seed, B=8):
    rng = np.random.default_rng(seed)
    params = [(W_ * 1.0, rng.standard_normal(b.shape) * 0.1) for W_, b in M.init_params(seed)]
    Xs = np.zeros((B, M.KIN))
    Xs[:, :M.NFEAT] = rng.standard_normal((B, M.NFEAT))
    T = rng.standard_normal((B, 3))
    return params, Xs, T


def test_gradients_match_central_differences():
    params, Xs, T = _small_problem(1)
    loss, grads = M.loss_and_grads(params, Xs, T, emulate=False)
    rng = np.random.default_rng(2)
    eps = 1e-6
    for l, (W_, b) in enumerate(params):
        for which, arr, g in (("W", W_, grads[l][0]), ("b", b, grads[l][1])):
            for _ in range(6):
                ix = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[ix]
                arr[ix] = old + eps
                lp, _ = M.loss_and_grads(params, Xs, T, emulate=False)
                arr[ix] = old - eps
                lm, _ = M.loss_and_grads(params, Xs, T, emulate=False)
                arr[ix] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(g[ix] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (l, which, ix, g[ix], fd)


def test_emulated_gradients_close_to_exact():
    # BF16 rounding at the product inputs perturbs the gradients by ~2^-9
    params, Xs, T = _small_problem(3, B=64)
    _, g0 = M.loss_and_grads(params, Xs, T, emulate=False)
    _, g1 = M.loss_and_grads(params, Xs, T, emulate=True)
    for (a, b), (c, d) in zip(g0, g1):
        assert np.linalg.norm(a - c) <= 2e-2 * np.linalg.norm(a)
        assert np.linalg.norm(b - d) <= 2e-2 * np.linalg.norm(b)


def test_zero_weights_give_output_bias():
    params, Xs, _ = _small_problem(4)
    params = [(np.zeros_like(W_), b) for W_, b in params]
    Y, _ = M.forward(params, Xs)
    np.testing.assert_array_equal(Y, np.broadcast_to(params[-1][1], Y.shape))


def test_adam_two_steps_by_hand():
    p0 = [(np.array([[1.0, -2.0]]), np.array([0.5, 0.0]))]
    g1 = [(np.array([[0.1, -0.3]]), np.array([2.0, 0.0]))]
    g2 = [(np.array([[-0.2, -0.1]]), np.array([1.0, 1e-3]))]
    opt = M.Adam(p0, lr=1e-3)
    p1 = opt.step(p0, g1)
    # step 1: m_hat = g, v_hat = g^2, update lr * g / (|g| + eps)
    np.testing.assert_allclose(p1[0][0], [[1.0 - 1e-3 * 0.1 / (0.1 + 1e-8), -2.0 + 1e-3 * 0.3 / (0.3 + 1e-8)]],
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(p1[0][1], [0.5 - 1e-3 * 2.0 / (2.0 + 1e-8), 0.0], rtol=0, atol=1e-15)
    p2 = opt.step(p1, g2)
    # step 2 for the first weight: m = 0.9*0.01 + 0.1*(-0.2) ... written out
    m = 0.9 * (0.1 * 0.1) + 0.1 * (-0.2)
    v = 0.999 * (0.001 * 0.01) + 0.001 * 0.04
    mh, vh = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    want = p1[0][0][0, 0] - 1e-3 * mh / (math.sqrt(vh) + 1e-8)
    assert abs(p2[0][0][0, 0] - want) < 1e-15


def test_training_loop_fits_linear_map():
    # a target that is a fixed linear map of the inputs: loss must fall 100-fold
    rng = np.random.default_rng(5)
    B = 256
    Xs = np.zeros((B, M.KIN))
    Xs[:, :M.NFEAT] = rng.standard_normal((B, M.NFEAT))
    A = rng.standard_normal((M.NFEAT, 3)) / math.sqrt(M.NFEAT)
    T = Xs[:, :M.NFEAT] @ A
    params = M.init_params(6)
    opt = M.Adam(params, lr=1e-3)
    l0, _ = M.loss_and_grads(params, Xs, T)
    for _ in range(300):
        loss, g = M.loss_and_grads(params, Xs, T)
        params = opt.step(params, g)
    assert loss < l0 / 100, (l0, loss)


def test_features_affine_and_constant_fields():
    nb = (6, 5, 7)
    box = (1.2, 1.0, 1.4)
    h = np.array(box) / np.array(nb)
    ncell = int(np.prod(nb))
    k, j, i = np.meshgrid(*[np.arange(v) for v in nb[::-1]], indexing="ij")
    xc = np.stack([(i.ravel() + 0.5) * h[0], (j.ravel() + 0.5) * h[1], (k.ravel() + 0.5) * h[2]])
    a = np.array([0.3, -1.1, 2.0])
    eps = np.full(ncell, 0.7)
    U = np.stack([1.0 + a @ xc, -2.0 + 0 * a @ xc, 0.5 * (a @ xc)])
    G = np.stack([np.full(ncell, 3.0)] * 3)
    rng = np.random.default_rng(7)
    # interior cells only: no clamping
    pos = np.stack([rng.uniform(h[a_], box[a_] - h[a_], 50) for a_ in range(3)], axis=1)
    d = rng.uniform(0.01, 0.04, 50)
    X = M.features(pos, d, eps, U, G, box, nb, prec32=False)
    ix = np.floor(pos / h).astype(int)
    col = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx, dy, dz) == (0, 0, 0):
                    xcen = (ix + 0.5) * h
                    np.testing.assert_allclose(X[:, col], 0.7)
                    np.testing.assert_allclose(X[:, col + 1], 1.0 + xcen @ a, rtol=1e-12)
                    np.testing.assert_allclose(X[:, col + 2], -2.0)
                    np.testing.assert_allclose(X[:, col + 4:col + 7], 3.0)
                else:
                    step = a @ (np.array([dx, dy, dz]) * h)
                    np.testing.assert_allclose(X[:, col], 0.0, atol=1e-15)
                    np.testing.assert_allclose(X[:, col + 1], step, rtol=1e-9, atol=1e-14)
                    np.testing.assert_allclose(X[:, col + 2], 0.0, atol=1e-14)
                    np.testing.assert_allclose(X[:, col + 3], 0.5 * step, rtol=1e-9, atol=1e-14)
                    np.testing.assert_allclose(X[:, col + 4:col + 7], 0.0, atol=1e-15)
                col += 7
    np.testing.assert_allclose(X[:, 189:192], pos / h - ix, rtol=0, atol=1e-12)
    np.testing.assert_allclose(X[:, 192], d / h[0], rtol=1e-15)
    # a particle at a cell centre has offsets 1/2; at a wall the outward
    # neighbours are clamped onto the centre, so their differences vanish
    p0 = np.array([[0.5 * h[0], 0.5 * h[1], 0.5 * h[2]]])
    X0 = M.features(p0, [0.02], eps, U, G, box, nb, prec32=False)
    np.testing.assert_allclose(X0[0, 189:192], 0.5, rtol=1e-15)
    assert np.all(X0[0, 0:7] == 0.0)          # (dx, dy, dz) = (-1, -1, -1) clamps to the centre


def _fields_at(fine_fn, grid, pos):
    import oracle
    fine = fine_fn(grid)
    rr = oracle.restrict_all(fine, grid)
    uF = np.stack([oracle.interp(f, grid.nf, grid.box, pos) for f in fine[:3]], axis=1)
    uB = np.stack([oracle.interp(rr["U"][a], grid.nb, grid.box, pos) for a in range(3)], axis=1)
    return uF, uB


def test_affine_field_has_zero_residual():
    # trilinear interpolation and cell averaging are exact for affine fields, so
    # away from the walls (where the bulk interpolation is clamped) the fine
    # lookup and the bulk interpolation agree
    grid = W.Grid((1.0, 1.0, 1.0), (8, 8, 8), 4)
    a = np.array([[0.3, -0.7, 1.1], [2.0, 0.1, -0.4], [0.0, 0.5, 0.25]])

    def fine_fn(g):
        xs = [(np.arange(n) + 0.5) * (L / n) for n, L in zip(g.nf, g.box)]
        Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
        return [1.0 + a[c, 0] * X + a[c, 1] * Y + a[c, 2] * Z for c in range(3)] + [X + Y]

    rng = np.random.default_rng(8)
    hb = 1.0 / 8
    pos = rng.uniform(0.5 * hb, 1 - 0.5 * hb, (2000, 3))
    uF, uB = _fields_at(fine_fn, grid, pos)
    R = M.residual_target(uF, uB)
    assert np.abs(R).max() < 1e-13
    # next to a wall it is not zero (the bulk interpolation is flat there)
    pw = np.array([[0.2 * hb, 0.5, 0.5]])
    uF, uB = _fields_at(fine_fn, grid, pw)
    assert abs(M.residual_target(uF, uB)[0, 0] - 0.3 * (0.2 * hb - 0.5 * hb)) < 1e-12


@pytest.mark.parametrize("name,lo,hi", [("cube64_cic", 4.5e-3, 7.5e-3)])
def test_bulk_interpolation_error_taylor_green(name, lo, hi):
    """Relative L2 error of bulk trilinear interpolation against the fine-grid
    lookup on the 64^3 / 256^3 Taylor-Green workload: the error the surrogate has
    to beat (measured ~5.7e-3 on 2e5 random points)."""
    w = W.WORKLOADS[name]
    rng = np.random.default_rng(9)
    pos = rng.random((200_000, 3)) * np.array(w.grid.box)
    uF, uB = _fields_at(lambda g: [np.asarray(f, np.float64) for f in W.fine_fields(w)], w.grid, pos)
    e = np.linalg.norm(uB - uF) / np.linalg.norm(uF)
    assert lo < e < hi, e


def test_target_scale_floor():
    R = np.zeros((10, 3))
    R[:, 0] = np.arange(10)
    R[:, 1] = np.arange(10) * 2
    s = M.target_scale(R)
    assert s[2] == s[1] and s[1] == pytest.approx(2 * s[0])
    np.testing.assert_array_equal(M.target_scale(np.zeros((4, 3))), [1.0, 1.0, 1.0])


def test_norm_stats_floors():
    rng = np.random.default_rng(10)
    X = rng.standard_normal((500, M.NFEAT))
    X[:, 7 * 13 + 5] *= 100.0                      # centre value of channel 5, std ~100
    X[:, 7 * 14 + 5] = rng.standard_normal(500) * 1e-9   # a neighbour difference that is rounding noise
    X[:, 192] = 0.02                               # constant feature
    mean, std = M.norm_stats(X)
    assert std[7 * 14 + 5] == pytest.approx(1e-4 * X[:, 7 * 13 + 5].std())
    assert std[192] == 1.0
    np.testing.assert_allclose(std[:7], X[:, :7].std(axis=0))   # unaffected where the spread is real
    np.testing.assert_allclose(mean, X.mean(axis=0))
