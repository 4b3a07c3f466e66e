"""GPU parity on the full-size workloads: many advected steps on the 64^3/256^3
grids, the 10-million-particle packed bed compared on samples, and the precision
study (compensated FP32 vs naive FP32 vs FP64 on the GPU) on its 2M subsample."""
import json
import os

import numpy as np
import pytest

import workload as W
from parity_util import (TOL_FP32_FIELD, TOL_FP64_FIELD, TOL_NAIVE, cfg_for, compare_step, emax, results_dir,
                         rms_rel, run_gpu, to_dev)

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


def _gpu_step_outputs(cpl, out, P, V):
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()
         if not k.startswith("fine")}
    g["diag_d"] = cpl.diag_dict(out["diag"])
    g["pos_new"] = P.cpu().numpy()
    g["vel_new"] = V.cpu().numpy()
    return g


def _advected_run(env, n, checked_steps, label):
    """Run the 64^3 / 256^3 Taylor-Green workload for its 100 explicit-Euler steps
    of dt = 1e-4 (drag the only force) on the GPU.  Before every step in
    ``checked_steps`` the GPU's own FP32 state (positions, velocities) is handed to
    the oracle, so that both sides bin identical inputs; that step's outputs are
    then compared element by element: cell, perm, count and start bit for bit for
    every particle; phi, U, P, grad P, F_fpi, drag, beta and the advected
    positions and velocities at e_max <= 1e-4; the FP64 sums at rel 1e-6."""
    torch, cpl, oracle = env
    w = W.WORKLOADS["cube64_cic"]
    pos, d, vel = W.particles(w, n=n)
    fine = W.fine_fields(w)
    fine64 = [np.ascontiguousarray(f, dtype=np.float64) for f in fine]
    cfg = cfg_for(cpl, w, pos.shape[0], advect=True, dt=w.dt)
    dev = "cuda:0"
    P, V, D = to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev)
    Fd = [to_dev(f, torch, dev) for f in fine]
    c = cpl.Coupler(cfg)
    rr = oracle.restrict_all(fine64, w.grid)
    # the oracle's independent per-particle loops on the host's cores (its
    # results do not depend on the thread count)
    prev = oracle.set_threads(min(16, len(os.sched_getaffinity(0))))
    checked = 0
    for k in range(w.steps):
        check = k in checked_steps
        if check:
            gp, gv = P.cpu().numpy(), V.cpu().numpy()
        out = c.step(P, V, D, Fd)
        torch.cuda.synchronize()
        if not check:
            continue
        g = _gpu_step_outputs(cpl, out, P, V)
        o = oracle.step(gp, gv, d, fine64, w.grid, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p, eps_min=w.eps_min,
                        cic=True, prec32=True, vel_source="fine", advect_dt=w.dt, fine_out="none", restricted=rr)
        errs = compare_step(g, o, pos.shape[0], w.grid.nb, w.grid.ratio, box=w.grid.box, fp64=False,
                            check_fine=False, label=f"{label} step {k}")
        checked += 1
        if k % 20 == 0 or k == w.steps - 1 or n > 500_000:
            print(f"{label} step {k}: e_max " + ", ".join(f"{a} {b:.1e}" for a, b in errs.items()), flush=True)
    c.close()
    oracle.set_threads(prev)
    assert checked == len(checked_steps)


def test_cube64_advected_steps(env):
    """Every one of the 100 advected steps on 200,000 particles (the oracle takes
    about half a second per step at this size), each from the GPU's own state."""
    _advected_run(env, 200_000, set(range(100)), "cube64 200k")


def test_cube64_advected_full_size(env):
    """The workload at its full 2,000,000 particles: all 100 steps run on the GPU,
    and six of them (first, second, three in between, last) are compared with the
    oracle run from the GPU's state before the step (about 5 s each)."""
    _advected_run(env, 2_000_000, {0, 1, 33, 66, 98, 99}, "cube64 2M")


def _bed_inputs(w):
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    return pos, d, vel, fine


def test_bed128_full_size_sampled(env):
    """The 10M-particle bed at full size (512x512x1024 fine cells), in the launch
    configuration the benchmark times.  Every bulk and particle output is compared
    with the oracle; the fine-grid outputs on 200,000 sampled fine cells."""
    torch, cpl, oracle = env
    w = W.WORKLOADS["bed128_cic"]
    pos, d, vel, fine = _bed_inputs(w)
    n = pos.shape[0]
    cfg = cfg_for(cpl, w, n)
    print(f"case bed128 n={n}", flush=True)
    dev = "cuda:0"
    P, V, D = to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev)
    Fd = [to_dev(f, torch, dev) for f in fine]
    c = cpl.Coupler(cfg)
    out = c.step(P, V, D, Fd)
    torch.cuda.synchronize()
    sample = np.random.default_rng(11).integers(0, w.grid.n_fine, 200_000)
    si = torch.from_numpy(sample).to(dev)
    g = {k: (v.cpu().numpy() if v is not None and not k.startswith("fine") else None) for k, v in out.items()}
    g["fine_eps"] = out["fine_eps"].reshape(-1)[si].cpu().numpy()
    g["fine_F"] = out["fine_F"].reshape(3, -1)[:, si].cpu().numpy()
    g["diag_d"] = cpl.diag_dict(out["diag"])
    c.close()
    del P, V, D, Fd
    torch.cuda.empty_cache()
    o = oracle.step(pos, vel, d, fine, w.grid, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p, eps_min=w.eps_min,
                    cic=True, prec32=True, vel_source="fine", fine_out="sample", fine_sample=sample)
    errs = compare_step(g, o, n, w.grid.nb, w.grid.ratio, box=w.grid.box, fp64=False,
                        fine_sample=np.arange(sample.size), label="bed128",
                        fine_sample_index=sample)
    print("bed128 e_max:", {k: f"{v:.2e}" for k, v in errs.items()})


def test_bed128_semi_implicit_two_fluid_full_size_sampled(env):
    """The 10M-particle bed at full size with the semi-implicit split and the
    two-fluid drag on (the benchmark's variant legs, both at once): every bulk
    and particle output, K, KU and the restricted alpha against the oracle; the
    fine-grid outputs (eps, F, K, KU) on 200,000 sampled fine cells."""
    torch, cpl, oracle = env
    from parity_util import emax, fine_scale_from_bulk, neighbourhood_max
    w = W.WORKLOADS["bed128_cic"]
    pos, d, vel, fine = _bed_inputs(w)
    alpha = W.fine_alpha(w)
    n = pos.shape[0]
    cfg = cfg_for(cpl, w, n)
    cfg.semi_implicit, cfg.vof, cfg.rho_f2, cfg.mu_f2 = 1, 1, 1.2, 1.8e-5
    print(f"case bed128 semi-implicit + two-fluid n={n}", flush=True)
    dev = "cuda:0"
    P, V, D = to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev)
    Fd = [to_dev(f, torch, dev) for f in fine]
    A = to_dev(alpha, torch, dev)
    c = cpl.Coupler(cfg)
    out = c.step(P, V, D, Fd, alpha=A)
    torch.cuda.synchronize()
    sample = np.random.default_rng(12).integers(0, w.grid.n_fine, 200_000)
    si = torch.from_numpy(sample).to(dev)
    g = {k: (v.cpu().numpy() if v is not None and not k.startswith("fine") else None) for k, v in out.items()}
    g["fine_eps"] = out["fine_eps"].reshape(-1)[si].cpu().numpy()
    g["fine_F"] = out["fine_F"].reshape(3, -1)[:, si].cpu().numpy()
    g["fine_K"] = out["fine_K"].reshape(-1)[si].cpu().numpy()
    g["fine_KU"] = out["fine_KU"].reshape(3, -1)[:, si].cpu().numpy()
    g["diag_d"] = cpl.diag_dict(out["diag"])
    c.close()
    del P, V, D, Fd, A, out
    torch.cuda.empty_cache()
    o = oracle.step(pos, vel, d, fine, w.grid, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p, eps_min=w.eps_min,
                    cic=True, prec32=True, vel_source="fine", fine_out="sample", fine_sample=sample,
                    semi_implicit=True, alpha=alpha, rho2=1.2, mu2=1.8e-5)
    nb, r = w.grid.nb, w.grid.ratio
    errs = compare_step(g, o, n, nb, r, box=w.grid.box, fp64=False, fine_sample=np.arange(sample.size),
                        label="bed128 semi+vof", fine_sample_index=sample)
    nc = int(np.prod(nb))
    errs.update({
        "alpha": emax(g["bulk_alpha"].ravel(), o["alpha"], field_scale=1.0),
        "K": emax(g["bulk_K"].ravel(), o["K"]),
        "KU": emax(g["bulk_KU"].reshape(3, nc), o["KU"], o["KU_mag"]),
        "fine_K": emax(g["fine_K"], o["fine_K"],
                       fine_scale_from_bulk(neighbourhood_max(np.abs(o["K"]), nb), nb, r, sample)),
        "fine_KU": emax(g["fine_KU"], o["fine_KU"],
                        fine_scale_from_bulk(neighbourhood_max(o["KU_mag"], nb), nb, r, sample)),
    })
    print("bed128 semi+vof e_max:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= TOL_FP32_FIELD
    dg, od = g["diag_d"], o["diag"]
    assert abs(dg["K_p"] - od["K_p"]) <= 1e-6 * od["K_p"]
    assert abs(dg["K_b"] - dg["K_p"]) <= 1e-6 * od["K_p"]
    assert abs(dg["K_f"] - dg["K_b"]) <= 1e-6 * od["K_p"]


def test_precision_study_bed128_sub2m(env, tmp_path):
    """The four precision modes on the GPU, each against the FP64 oracle, on the
    2M-particle subsample of the bed (same grids): FP32 with Kahan-compensated
    FP32 per-cell sums, FP32 with FP64 register per-cell sums (the default FP32
    mode), naive FP32 and FP64; per-field max and RMS error, and the
    conservation residuals of the FP64 global sums."""
    torch, cpl, oracle = env
    w = W.WORKLOADS["bed128_sub2m"]
    pos, d, vel, fine = _bed_inputs(w)
    n = pos.shape[0]
    sample = np.random.default_rng(12).integers(0, w.grid.n_fine, 200_000)
    o = oracle.step(pos, vel, d, fine, w.grid, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p, eps_min=w.eps_min,
                    cic=True, prec32=True, vel_source="fine", fine_out="sample", fine_sample=sample)
    dev = "cuda:0"
    report = {}
    for mode, prec in (("fp32_kahan", cpl.COUPLE_FP32_KAHAN), ("fp32_wide", cpl.COUPLE_FP32_WIDE),
                       ("fp32_naive", cpl.COUPLE_FP32_NAIVE), ("fp64", cpl.COUPLE_FP64)):
        cfg = cfg_for(cpl, w, n, precision=prec)
        dt = cfg.dtype
        print(f"case precision {mode}", flush=True)
        P, V, D = to_dev(pos, torch, dev, dt), to_dev(vel, torch, dev, dt), to_dev(d, torch, dev, dt)
        Fd = [to_dev(f, torch, dev, dt) for f in fine]
        c = cpl.Coupler(cfg)
        out = c.step(P, V, D, Fd)
        torch.cuda.synchronize()
        si = torch.from_numpy(sample).to(dev)
        g = {k: (v.cpu().numpy() if v is not None and not k.startswith("fine") else None) for k, v in out.items()}
        g["fine_eps"] = out["fine_eps"].reshape(-1)[si].cpu().numpy()
        g["fine_F"] = out["fine_F"].reshape(3, -1)[:, si].cpu().numpy()
        g["diag_d"] = cpl.diag_dict(out["diag"])
        c.close()
        del P, V, D, Fd, out
        torch.cuda.empty_cache()
        errs = compare_step(g, o, n, w.grid.nb, w.grid.ratio, box=w.grid.box, fp64=(mode == "fp64"),
                            naive=(mode == "fp32_naive"), fine_sample=np.arange(sample.size),
                            label=mode, fine_sample_index=sample)
        rms = {"phi": rms_rel(g["bulk_phi"], o["phi"]), "U": rms_rel(g["bulk_U"], o["U"]),
               "P": rms_rel(g["bulk_P"], o["P"]), "G": rms_rel(g["bulk_G"], o["G"]),
               "F": rms_rel(g["bulk_F"], o["F"]), "drag": rms_rel(g["drag"], o["drag"]),
               "beta": rms_rel(g["beta"], o["beta"]), "fine_eps": rms_rel(g["fine_eps"], o["fine_eps"]),
               "fine_F": rms_rel(g["fine_F"], o["fine_F"])}
        dg = g["diag_d"]
        sabs = np.abs(o["drag"]).sum(axis=0)
        report[mode] = {
            "e_max": errs, "rms_rel": rms,
            "V_dep/V_tot - 1": dg["V_dep"] / dg["V_tot"] - 1.0,
            "(S_b + sum F_p) / sum|F_p|": [(dg["S_b"][a] + dg["sum_Fp"][a]) / sabs[a] for a in range(3)],
            "(S_f - S_b) / sum|F_p|": [(dg["S_f"][a] - dg["S_b"][a]) / sabs[a] for a in range(3)],
        }
    os.makedirs(results_dir(), exist_ok=True)
    with open(os.path.join(results_dir(), "precision_study_bed128_sub2m.json"), "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps(report, indent=1))
    assert max(report["fp64"]["e_max"].values()) <= TOL_FP64_FIELD
    assert max(report["fp32_kahan"]["e_max"].values()) <= TOL_FP32_FIELD
    assert max(report["fp32_wide"]["e_max"].values()) <= TOL_FP32_FIELD
    assert max(report["fp32_naive"]["e_max"].values()) <= TOL_NAIVE
    # FP64 register sums keep the restricted U and P within about one FP32
    # rounding of the exact averages (2^-24 relative), and the pressure's low
    # word keeps the gradient there too.
    k = report["fp32_wide"]["e_max"]
    assert k["U"] <= 1.2e-7 and k["P"] <= 1.2e-7, k
    assert k["G"] <= 3e-7, k
    # The deposited fields are limited by the FP32 positions, diameters and drag
    # (a few roundings of each term), not by the sums: measured 2e-7 to 6e-7.
    assert k["phi"] <= 1e-6 and k["F"] <= 2e-6 and k["fine_eps"] <= 1e-6 and k["fine_F"] <= 2e-6, k
    # Kahan in FP32 bounds each per-cell sum by about two FP32 roundings of the
    # sum of magnitudes; the gradient differences two such averages over one
    # cell width, so it may lose a few more digits than U and P.
    kk = report["fp32_kahan"]["e_max"]
    assert kk["U"] <= 5e-7 and kk["P"] <= 5e-7 and kk["phi"] <= 2e-6 and kk["F"] <= 5e-6, kk


def test_bed128_surrogate_full_size_sampled(env):
    """The surrogate step on the 10M-particle bed in the benchmark's launch
    configuration (vel_source MLP, no fallback): on 20,000 sampled particles the
    network part of the velocity matches the BF16-emulating oracle network fed
    with the features of the GPU's own bulk fields; the bulk fields equal the
    plain step's."""
    torch, cpl, oracle = env
    from oracle import mlp as M
    w = W.WORKLOADS["bed128_cic"]
    pos, d, vel = W.particles(w)
    n = pos.shape[0]
    dev = "cuda:0"
    P, V, D = to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev)
    Fd = W.fine_fields_torch(w, dev, torch.float32)
    cfg = cfg_for(cpl, w, n)
    print("case bed128 surrogate: plain step", flush=True)
    c = cpl.Coupler(cfg)
    out = c.step(P, V, D, Fd, uf=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)

    def feats(ids):
        S = torch.from_numpy(ids.astype(np.int32)).to(dev)
        f = torch.empty((ids.size, 193), dtype=torch.float32, device=dev)
        ub = torch.empty((ids.size, 3), dtype=torch.float32, device=dev)
        r = torch.empty((ids.size, 3), dtype=torch.float32, device=dev)
        cpl.couple_mlp_features(cfg, P, D, out["bulk_phi"], out["bulk_U"], out["bulk_G"], f, u_fine=out["uf"],
                                sel=S, u_bulk=ub, resid=r)
        torch.cuda.synchronize()
        return f.cpu().numpy().astype(np.float64), ub.cpu().numpy().astype(np.float64), r.cpu().numpy()

    X, _, R = feats(rng.choice(n, 200_000, replace=False))
    mean, std = M.norm_stats(X)
    scale = M.target_scale(R)
    rp = np.random.default_rng(1013)
    params = [(Wl, rp.standard_normal(b.shape) * 0.2) for Wl, b in M.init_params(13)]
    net = cpl.Mlp(1024)
    net.set_params(M.flatten(params))
    net.set_norm(mean, std, scale)
    cm = cpl.Config(**{**cfg.__dict__, "vel_source": cpl.COUPLE_VEL_MLP, "mlp_tol": 1e30})
    h = cpl.Coupler(cm)
    cpl.couple_set_mlp(h.h, net.m)
    print("case bed128 surrogate: surrogate step", flush=True)
    om = h.step(P, V, D, Fd, uf=True, step=3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(om["bulk_U"].cpu().numpy(), out["bulk_U"].cpu().numpy())
    np.testing.assert_array_equal(om["bulk_phi"].cpu().numpy(), out["bulk_phi"].cpu().numpy())
    assert cpl.diag_dict(om["diag"])["n_fallback"] == 0
    ids = rng.choice(n, 20_000, replace=False)
    Xs, ubs, _ = feats(ids)
    Y, _ = M.forward(params, M.standardise(Xs, mean, std), emulate=True)
    g = om["uf"].cpu().numpy()[ids].astype(np.float64)
    e = float(np.linalg.norm(g - ubs - Y * scale) / np.linalg.norm(Y * scale))
    # per particle as well (a wrong or misplaced row would hide in the norm): the
    # in-step bound of tests/test_gpu_mlp.py, |d| <= 1e-2 max(|y|, rms/2) (its
    # inputs are standardised in FP32 in the step, in FP64 here)
    part, ref = g - ubs, Y * scale
    rn = np.linalg.norm(ref, axis=1)
    er = np.linalg.norm(part - ref, axis=1) / np.maximum(rn, 0.5 * np.sqrt(np.mean(rn ** 2)))
    print(f"bed128 surrogate, network part on 20,000 samples: rel {e:.2e}, worst row {er.max():.2e}", flush=True)
    assert er.max() <= 1e-2, (int(er.argmax()), float(er.max()))
    h.close()
    c.close()
    net.close()
    assert e <= 1e-3
