"""GPU parity of the learned velocity surrogate against its FP64 oracle
(oracle/mlp.py, BF16 rounding emulated at the same points): features, forward,
gradients, Adam, checkpoint/resume, the in-step inference with its sampled check
and fine fallback, and the drag computed from the surrogate's velocity."""
import numpy as np
import pytest

import workload as W
from oracle import mlp as M
from parity_util import TOL_FP32_FIELD, cfg_for, compare_step, to_dev

pytestmark = pytest.mark.gpu

TOL_MLP = 1e-3   # norm-wise relative error of network outputs and gradients
# Per particle: |y_gpu - y_oracle| <= TOL_ROW * max(|y_oracle|, 1e-2 rms|y_oracle|).
# The two sides round to BF16 at the same points but accumulate in FP32 and FP64;
# where an activation lies within an FP32 rounding of a BF16 rounding boundary
# the two roundings differ by one BF16 step (2^-8 relative) in that activation,
# whose effect on an output row is a fraction of that step: 1e-2 bounds a row
# with several such flips, and catches a wrong or misplaced row (an error of
# order one).
TOL_ROW = 1e-2
# In the step the network's inputs are gathered and standardised by the inference
# kernel in FP32, while the reference features are standardised in FP64: an input
# within one FP32 rounding of a BF16 rounding boundary then rounds to the other
# BF16 neighbour on the two sides (one input in ~2^16), changing that input by one
# BF16 step (2^-8 of a standardised value of at most a few units) and the row's
# output by a few 1e-3 of the output scale.  The in-step rows are therefore held
# to TOL_ROW relative to max(|y|, rms/2): a row whose network part is wrong or
# misplaced, or off by 10 % of a typical row, still fails.
ROW_FLOOR_INSTEP = 0.5


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _assert_rows(got, ref, label, tol=TOL_ROW, floor_frac=1e-2):
    """Per-row bound above, on [n, k] outputs: |g - o| <= tol * max(|o|,
    floor_frac * rms |o|); returns the worst row's error."""
    g = np.asarray(got, np.float64).reshape(len(ref), -1)
    o = np.asarray(ref, np.float64).reshape(len(ref), -1)
    rn = np.linalg.norm(o, axis=1)
    floor = floor_frac * np.sqrt(np.mean(rn ** 2)) if rn.size else 0.0
    err = np.linalg.norm(g - o, axis=1) / np.maximum(np.maximum(rn, floor), 1e-300)
    worst = float(err.max()) if err.size else 0.0
    assert worst <= tol, f"{label}: row {int(err.argmax())} error {worst:.3e} > {tol}"
    return worst


def _params(seed, bias_scale=0.05):
    rng = np.random.default_rng(seed + 1000)
    return [(Wl, rng.standard_normal(b.shape) * bias_scale) for Wl, b in M.init_params(seed)]


def _small_case(torch, cpl, nb=(12, 10, 14), n=20000, seed=21):
    """A FINE-velocity step on a small Taylor-Green workload; returns host and device data."""
    w = W.small_workload(nb=nb, ratio=4, box=(1.2, 1.0, 1.4), n=n, seed=seed, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    dev = "cuda:0"
    cfg = cfg_for(cpl, w, n)
    P, V, D = to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev)
    Fd = [to_dev(f, torch, dev) for f in fine]
    c = cpl.Coupler(cfg)
    out = c.step(P, V, D, Fd, uf=True)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    c.close()
    return dict(w=w, cfg=cfg, pos=pos, d=d, vel=vel, fine=fine, P=P, V=V, D=D, Fd=Fd, out=out, host=host)


def _features(torch, cpl, case, sel=None):
    dev = "cuda:0"
    n = case["pos"].shape[0]
    m = n if sel is None else len(sel)
    feat = torch.empty((m, 193), dtype=torch.float32, device=dev)
    ub = torch.empty((m, 3), dtype=torch.float32, device=dev)
    res = torch.empty((m, 3), dtype=torch.float32, device=dev)
    S = None if sel is None else torch.from_numpy(np.asarray(sel, np.int32)).to(dev)
    o = case["out"]
    cpl.couple_mlp_features(case["cfg"], case["P"], case["D"], o["bulk_phi"], o["bulk_U"], o["bulk_G"], feat,
                            u_fine=o["uf"], sel=S, u_bulk=ub, resid=res)
    torch.cuda.synchronize()
    return feat, ub, res


def test_features_match_oracle(env):
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    h, g = case["host"], case["w"].grid
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    # the oracle's features of the GPU's own bulk fields (the same FP32 inputs)
    phi = h["bulk_phi"].astype(np.float64).ravel()
    U = h["bulk_U"].astype(np.float64).reshape(3, -1)
    G = h["bulk_G"].astype(np.float64).reshape(3, -1)
    Xo = M.features(case["pos"], case["d"], 1.0 - phi, U, G, g.box, g.nb, prec32=True)
    # stencil values: FP32 differences of FP32 inputs (one rounding; eps = 1 - phi
    # adds one rounding of size ulp(1)/2 per operand); offsets x n / L - i: one
    # FP32 product of size up to n (its ulp)
    tol = 1e-6 * (np.abs(Xo).max(axis=0) + 1e-30)
    tol[0:189:7] = np.maximum(tol[0:189:7], 2.0 ** -22)
    tol[189:192] = 2.0 ** -22 * np.asarray(g.nb, np.float64)
    err = np.abs(X - Xo) / tol
    assert err.max() <= 1.0, (err.max(), int(np.argmax(err.max(axis=0))))
    # bulk interpolation and residual
    uB = np.stack([oracle.interp(U[a], g.nb, g.box, case["pos"], True) for a in range(3)], axis=1)
    assert np.abs(ub.cpu().numpy() - uB).max() <= 1e-6 * np.abs(uB).max()
    np.testing.assert_array_equal(res.cpu().numpy(), (h["uf"] - ub.cpu().numpy()).astype(np.float32))
    # selected rows equal the full computation bitwise
    sel = np.random.default_rng(3).choice(case["pos"].shape[0], 777, replace=False)
    f2, u2, r2 = _features(torch, cpl, case, sel)
    np.testing.assert_array_equal(f2.cpu().numpy(), X[sel].astype(np.float32))
    np.testing.assert_array_equal(r2.cpu().numpy(), res.cpu().numpy()[sel])


def _net(torch, cpl, params, mean, std, scale, max_batch=4096):
    m = cpl.Mlp(max_batch)
    m.set_params(M.flatten(params))
    m.set_norm(mean, std, scale)
    return m


def test_forward_matches_oracle(env):
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    params = _params(1)
    m = _net(torch, cpl, params, mean, std, [1.0, 1.0, 1.0])
    n = 3001   # several 16-row tiles and a ragged tail
    y = torch.empty((n, 3), dtype=torch.float32, device="cuda:0")
    m.forward(feat[:n].contiguous(), y)
    torch.cuda.synchronize()
    Yo, _ = M.forward(params, M.standardise(X[:n], mean, std), emulate=True)
    yg = y.cpu().numpy()
    e = _rel(yg, Yo)
    # every row, and the last, partial 16-row tile (rows 2992..3000) on its own
    er = _assert_rows(yg, Yo, "forward")
    et = _assert_rows(yg[2992:], Yo[2992:], "forward, ragged tail")
    assert _rel(yg[2992:], Yo[2992:]) <= TOL_MLP
    print(f"forward rel err {e:.2e}; worst row {er:.2e}; ragged tail worst row {et:.2e}")
    assert e <= TOL_MLP
    # zero rows -> nothing to do
    m.forward(feat[:0], y[:0])
    m.close()


def test_gradients_match_oracle(env):
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    R = res.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    scale = M.target_scale(R)
    params = _params(2)
    m = _net(torch, cpl, params, mean, std, scale)
    B = 1024
    idx = np.random.default_rng(4).choice(X.shape[0], B, replace=False).astype(np.int32)
    grads = torch.empty(M.NPARAM, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    m.grads(feat, res, B, grads, idx=torch.from_numpy(idx).cuda(), loss=loss)
    torch.cuda.synchronize()
    lo, go = M.loss_and_grads(params, M.standardise(X[idx], mean, std), R[idx] / scale, emulate=True)
    assert abs(float(loss.item()) - lo) <= 1e-4 * lo, (loss.item(), lo)
    gg = M.unflatten(grads.cpu().numpy())
    for l, ((gw, gb), (ow, ob)) in enumerate(zip(gg, go)):
        ew, eb = _rel(gw, ow), _rel(gb, ob)
        print(f"layer {l}: dW rel {ew:.2e}, db rel {eb:.2e}")
        assert ew <= TOL_MLP and eb <= TOL_MLP
    # the gradient call leaves the parameters alone
    np.testing.assert_array_equal(m.get_state()["params"], M.flatten(params))
    m.close()


@pytest.mark.parametrize("B, use_idx", [(32, True), (96, False), (288, True), (4096, True)])
def test_gradients_at_edge_batch_sizes(env, B, use_idx):
    """Gradient parity where the batch leaves partial units: the training pass
    takes 32 rows per workgroup and the weight-gradient products 256-row chunks
    (one workgroup; a single partial chunk without an index; a whole chunk and
    a partial one; the largest batch of the handle)."""
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    R = res.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    scale = M.target_scale(R)
    params = _params(5)
    m = _net(torch, cpl, params, mean, std, scale)
    rows = (np.random.default_rng(B).choice(X.shape[0], B, replace=False).astype(np.int32) if use_idx
            else np.arange(B, dtype=np.int32))
    grads = torch.empty(M.NPARAM, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    m.grads(feat, res, B, grads, idx=torch.from_numpy(rows).cuda() if use_idx else None, loss=loss)
    torch.cuda.synchronize()
    lo, go = M.loss_and_grads(params, M.standardise(X[rows], mean, std), R[rows] / scale, emulate=True)
    assert abs(float(loss.item()) - lo) <= 1e-4 * lo, (loss.item(), lo)
    gg = M.unflatten(grads.cpu().numpy())
    for l, ((gw, gb), (ow, ob)) in enumerate(zip(gg, go)):
        ew, eb = _rel(gw, ow), _rel(gb, ob)
        print(f"B {B} layer {l}: dW rel {ew:.2e}, db rel {eb:.2e}")
        assert ew <= TOL_MLP and eb <= TOL_MLP, (B, l, ew, eb)
    m.close()


def test_gradients_with_out_of_range_indices_read_row_zero(env):
    """Batch indices outside [0, nrows) read row 0 (the documented guard that
    keeps every load in bounds): the gradients equal those of the same batch
    with such indices replaced by 0, bit for bit."""
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    R = res.cpu().numpy().astype(np.float64)
    m = _net(torch, cpl, _params(6), *M.norm_stats(X), M.target_scale(R))
    B = 96
    idx = np.random.default_rng(7).choice(X.shape[0], B, replace=False).astype(np.int32)
    bad = idx.copy()
    bad[[3, 40, 95]] = [-1, X.shape[0], 2 ** 31 - 1]
    fixed = bad.copy()
    fixed[(fixed < 0) | (fixed >= X.shape[0])] = 0
    out = []
    for ix in (bad, fixed):
        g = torch.empty(M.NPARAM, dtype=torch.float32, device="cuda:0")
        m.grads(feat, res, B, g, idx=torch.from_numpy(ix).cuda())
        torch.cuda.synchronize()
        out.append(g.cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])
    m.close()


def test_adam_matches_oracle(env):
    torch, cpl, oracle = env
    params = _params(3)
    m = _net(torch, cpl, params, np.zeros(193), np.ones(193), [1.0, 1.0, 1.0])
    rng = np.random.default_rng(5)
    opt = M.Adam(params, lr=1e-3)
    p = [(a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for a, b in params]
    for k in range(3):
        g = (rng.standard_normal(M.NPARAM) * 10.0 ** rng.uniform(-6, 0, M.NPARAM)).astype(np.float32)
        m.adam(torch.from_numpy(g).cuda())
        p = opt.step(p, M.unflatten(g))
    torch.cuda.synchronize()
    st = m.get_state()
    assert st["step"] == 3
    want = M.flatten(p).astype(np.float64)
    got = st["params"].astype(np.float64)
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-9)
    m.close()


def test_checkpoint_resume_is_bitwise(env):
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    m = cpl.Mlp(2048)
    m.set_params(M.flatten(_params(4)))
    m.fit_norm(feat, res)
    rng = np.random.default_rng(6)
    batches = [torch.from_numpy(rng.choice(feat.shape[0], 512, replace=False).astype(np.int32)).cuda()
               for _ in range(10)]
    for b in batches[:5]:
        m.train_step(feat, res, 512, idx=b)
    ck = m.get_state()
    for b in batches[5:]:
        m.train_step(feat, res, 512, idx=b)
    a = m.get_state()
    m2 = cpl.Mlp(2048)
    m2.set_state(ck)
    for b in batches[5:]:
        m2.train_step(feat, res, 512, idx=b)
    b2 = m2.get_state()
    for k in ("params", "m", "v", "mean", "std", "scale"):
        np.testing.assert_array_equal(a[k], b2[k], err_msg=k)
    assert a["step"] == b2["step"] == 10
    m.close()
    m2.close()


def test_fit_norm_matches_oracle(env):
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    m = cpl.Mlp(64)
    m.fit_norm(feat, res)
    st = m.get_state()
    X = feat.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    np.testing.assert_allclose(st["mean"], mean, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(st["std"], std, rtol=1e-10)
    np.testing.assert_allclose(st["scale"], M.target_scale(res.cpu().numpy()), rtol=1e-10)
    m.close()


def _mlp_step(torch, cpl, case, net, tol, period=100, step=0):
    cfg = cfg_for(cpl, case["w"], case["pos"].shape[0], vel_source=cpl.COUPLE_VEL_MLP)
    cfg.mlp_tol, cfg.mlp_period = tol, period
    c = cpl.Coupler(cfg)
    cpl.couple_set_mlp(c.h, net.m)
    out = c.step(case["P"], case["V"], case["D"], case["Fd"], uf=True, step=step)
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    host["diag_d"] = cpl.diag_dict(out["diag"])
    c.close()
    return host


def test_step_inference_matches_oracle(env):
    """vel_source MLP with no fallback: the velocity at every particle is
    u_bulk + s * y.  (1) Against the oracle's network on the features of the
    GPU's own bulk fields: the network part within 1e-3.  (2) Against the whole
    oracle pipeline (its own FP64 bulk fields): within 5e-3, the features now
    differing by ~1e-6 relative, which moves some BF16-rounded inputs by one
    BF16 step (measured 1.6e-3 with this untrained network).  (3) The rest of
    the step (drag, sources, prolongation, sums) matches the oracle run with the
    GPU's velocity."""
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    R = res.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    scale = M.target_scale(R)
    params = _params(5, bias_scale=0.2)
    net = _net(torch, cpl, params, mean, std, scale)
    g = _mlp_step(torch, cpl, case, net, tol=1e30)
    assert g["diag_d"]["n_fallback"] == 0
    ubg = ub.cpu().numpy().astype(np.float64)
    Yg, _ = M.forward(params, M.standardise(X, mean, std), emulate=True)
    e1 = _rel(g["uf"] - ubg, Yg * scale)
    w = case["w"]
    o = oracle.step(case["pos"], case["vel"], case["d"], case["fine"], w.grid, rho_f=w.rho_f, mu_f=w.mu_f,
                    rho_p=w.rho_p, eps_min=w.eps_min, cic=True, prec32=True, vel_source="bulk", fine_out="none")
    Xo = M.features(case["pos"], case["d"], 1.0 - o["phi"], o["U"], o["G"], w.grid.box, w.grid.nb)
    u_o = M.predict(params, Xo, mean, std, scale, o["uf"])
    e2 = _rel(g["uf"] - o["uf"], u_o - o["uf"])
    r1 = _assert_rows(g["uf"] - ubg, Yg * scale, "in-step network part", floor_frac=ROW_FLOOR_INSTEP)
    # against the whole oracle pipeline the BF16-rounded inputs themselves can
    # differ by a step (reported, bounded norm-wise)
    g2 = np.asarray(g["uf"] - o["uf"], np.float64)
    o2n = np.linalg.norm(u_o - o["uf"], axis=1)
    r2 = float((np.linalg.norm(g2 - (u_o - o["uf"]), axis=1) /
                np.maximum(o2n, 1e-2 * np.sqrt(np.mean(o2n ** 2)))).max())
    print(f"in-step surrogate, network part: vs oracle network on GPU fields {e1:.2e} (worst row {r1:.2e}), "
          f"vs oracle pipeline {e2:.2e} (worst row {r2:.2e})")
    assert e1 <= TOL_MLP and e2 <= 5 * TOL_MLP
    # the bulk fields are the plain path's
    np.testing.assert_array_equal(g["bulk_U"], case["host"]["bulk_U"])
    np.testing.assert_array_equal(g["bulk_G"], case["host"]["bulk_G"])
    # the rest of the step with the GPU's velocity
    o2 = oracle.step(case["pos"], case["vel"], case["d"], case["fine"], w.grid, rho_f=w.rho_f, mu_f=w.mu_f,
                     rho_p=w.rho_p, eps_min=w.eps_min, cic=True, prec32=True, vel_source="given",
                     bulk_velocity=g["uf"])
    compare_step(g, o2, case["pos"].shape[0], w.grid.nb, w.grid.ratio, fp64=False, box=w.grid.box, label="mlp step")
    net.close()


def test_step_with_semi_implicit_and_two_fluid_drag(env):
    """The options compose with the surrogate velocity: vel_source MLP with the
    semi-implicit split and the two-fluid drag on.  Everything after the
    velocity (drag with the mixed density and viscosity, sources, K and KU,
    prolongation, sums) matches the oracle run with the GPU's velocity."""
    torch, cpl, oracle = env
    case = _small_case(torch, cpl, seed=23)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    R = res.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    net = _net(torch, cpl, _params(6, bias_scale=0.2), mean, std, M.target_scale(R))
    w = case["w"]
    alpha = W.fine_alpha(w)
    cfg = cfg_for(cpl, w, case["pos"].shape[0], vel_source=cpl.COUPLE_VEL_MLP)
    cfg.mlp_tol, cfg.semi_implicit, cfg.vof, cfg.rho_f2, cfg.mu_f2 = 1e30, 1, 1, 1.2, 1.8e-5
    print("case mlp + semi-implicit + two-fluid", flush=True)
    c = cpl.Coupler(cfg)
    try:
        cpl.couple_set_mlp(c.h, net.m)
        out = c.step(case["P"], case["V"], case["D"], case["Fd"], uf=True, alpha=to_dev(alpha, torch, "cuda:0"))
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        g["diag_d"] = cpl.diag_dict(out["diag"])
    finally:
        c.close()
    o = oracle.step(case["pos"], case["vel"], case["d"], case["fine"], w.grid, rho_f=w.rho_f, mu_f=w.mu_f,
                    rho_p=w.rho_p, eps_min=w.eps_min, cic=True, prec32=True, vel_source="given",
                    bulk_velocity=g["uf"], semi_implicit=True, alpha=alpha, rho2=1.2, mu2=1.8e-5)
    nb, r = w.grid.nb, w.grid.ratio
    compare_step(g, o, case["pos"].shape[0], nb, r, fp64=False, box=w.grid.box, label="mlp+semi+vof")
    nc = int(np.prod(nb))
    from parity_util import emax, fine_scale_from_bulk, neighbourhood_max
    errs = {
        "alpha": emax(g["bulk_alpha"].ravel(), o["alpha"], field_scale=1.0),
        "K": emax(g["bulk_K"].ravel(), o["K"]),
        "KU": emax(g["bulk_KU"].reshape(3, nc), o["KU"], o["KU_mag"]),
        "fine_K": emax(g["fine_K"].ravel(), o["fine_K"],
                       fine_scale_from_bulk(neighbourhood_max(np.abs(o["K"]), nb), nb, r)),
        "fine_KU": emax(g["fine_KU"].reshape(3, -1), o["fine_KU"],
                        fine_scale_from_bulk(neighbourhood_max(o["KU_mag"], nb), nb, r)),
    }
    print("mlp + semi + vof e_max:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= TOL_FP32_FIELD
    net.close()


def _bricks_with_sample(cell, nb, period, phase):
    ids = np.arange(cell.size)
    c = cell.astype(np.int64)
    ix, iy, iz = c % nb[0], (c // nb[0]) % nb[1], c // (nb[0] * nb[1])
    bx, by = (nb[0] + 7) // 8, (nb[1] + 7) // 8
    brick = ix // 8 + bx * (iy // 8 + by * (iz // 8))
    sampled = np.unique(brick[ids % period == phase])
    return brick, sampled


def test_fallback_on_bad_network(env):
    """An untrained network fails the sampled check: every brick that holds a
    checked particle falls back to the fine lookup (the plain path's velocity),
    the others keep the network's; counts match."""
    torch, cpl, oracle = env
    case = _small_case(torch, cpl, nb=(20, 18, 17), n=30000)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    net = _net(torch, cpl, _params(6, bias_scale=1.0), mean, std, [0.1, 0.1, 0.1])
    period, step = 997, 5
    g = _mlp_step(torch, cpl, case, net, tol=1e-3, period=period, step=step)
    brick, sampled = _bricks_with_sample(case["host"]["cell"], case["w"].grid.nb, period, step % period)
    fell = np.isin(brick, sampled)
    d = g["diag_d"]
    assert d["n_fallback"] == fell.sum() and 0 < fell.sum() < fell.size
    assert d["mlp_nsamp"] == np.sum(np.arange(fell.size) % period == step % period)
    # the fallback is the plain path's trilinear lookup of the same fine values
    # (read from global memory there, from LDS in the plain kernel): equal to
    # FP32 rounding
    ulp = 2.0 ** -23 * np.abs(case["host"]["uf"]).max()
    np.testing.assert_allclose(g["uf"][fell], case["host"]["uf"][fell], rtol=0, atol=2 * ulp)
    assert np.all(np.any(g["uf"][~fell] != case["host"]["uf"][~fell], axis=1))
    # the sampled error the step reports is that of the network before fallback
    ids = np.arange(fell.size) % period == step % period
    pre = _mlp_step(torch, cpl, case, net, tol=1e30, period=period, step=step)["uf"].astype(np.float64)
    np.testing.assert_array_equal(pre[~fell], g["uf"][~fell])
    fine_u = case["host"]["uf"][ids].astype(np.float64)
    e2 = np.sum((pre[ids] - fine_u) ** 2)
    r2 = np.sum(fine_u ** 2)
    # (the check looks the fine velocity up itself; it agrees with the plain
    # path to FP32 rounding)
    assert abs(d["mlp_err2"] - e2) <= 1e-6 * e2 and abs(d["mlp_ref2"] - r2) <= 1e-6 * r2
    net.close()


def test_fallback_everywhere_with_zero_tolerance(env):
    torch, cpl, oracle = env
    case = _small_case(torch, cpl)
    feat, ub, res = _features(torch, cpl, case)
    X = feat.cpu().numpy().astype(np.float64)
    mean, std = M.norm_stats(X)
    net = _net(torch, cpl, _params(7), mean, std, M.target_scale(res.cpu().numpy()))
    g = _mlp_step(torch, cpl, case, net, tol=0.0, period=1)
    assert g["diag_d"]["n_fallback"] == case["pos"].shape[0]
    assert g["diag_d"]["mlp_nsamp"] == case["pos"].shape[0]
    ulp = 2.0 ** -23 * np.abs(case["host"]["uf"]).max()
    np.testing.assert_allclose(g["uf"], case["host"]["uf"], rtol=0, atol=2 * ulp)
    # the void fraction at the particle comes from another kernel (the compiler
    # may contract its products differently): equal to FP32 rounding
    np.testing.assert_allclose(g["drag"], case["host"]["drag"], rtol=1e-5, atol=1e-6 * np.abs(g["drag"]).max())
    net.close()


def test_mlp_mode_errors(env):
    torch, cpl, oracle = env
    w = W.small_workload(nb=(4, 4, 4), n=10, precision="fp32")
    cfg = cfg_for(cpl, w, 10, vel_source=cpl.COUPLE_VEL_MLP)
    c = cpl.Coupler(cfg)
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    dev = "cuda:0"
    with pytest.raises(cpl.CoupleError) as ei:
        c.step(to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev),
               [to_dev(f, torch, dev) for f in fine])
    assert ei.value.code == cpl.COUPLE_ESTATE
    c.close()
    m = cpl.Mlp(64)
    with pytest.raises(cpl.CoupleError):
        m.grads(torch.zeros((64, 193), device=dev), torch.zeros((64, 3), device=dev), 48,
                torch.empty(cpl.MLP_NPARAM, device=dev))       # not a multiple of 32
    with pytest.raises(cpl.CoupleError):
        m.forward(torch.zeros((65, 193), device=dev), torch.empty((65, 3), device=dev))   # > max_batch
    with pytest.raises(cpl.CoupleError):
        m.set_norm(np.zeros(193), np.zeros(193), [1, 1, 1])    # std must be > 0
    m.close()
