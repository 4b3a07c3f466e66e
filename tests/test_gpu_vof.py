"""GPU parity of the two-fluid (VOF) drag against the FP64 oracle, through the C
ABI: the fluid density and viscosity at each particle are mixed by the liquid
volume fraction (Sec. 2.5), restricted from the fine grid and interpolated
trilinearly to the particle.  The restricted alpha is compared element by
element (scale: the field's maximum, alpha being in [0, 1]); the drag, beta and
every downstream field through the usual step comparison."""
import numpy as np
import pytest

import workload as W
from parity_util import TOL_FP32_FIELD, TOL_FP64_FIELD, TOL_NAIVE, cfg_for, compare_step, emax, run_gpu

pytestmark = pytest.mark.gpu

RHO2, MU2 = 1.2, 1.8e-5


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


CASES = [
    # (nb, ratio, box, n, precision, deposit, vel_source, semi)
    ((5, 3, 4), 4, (1.0, 0.75, 1.25), 777, "fp32w", "cic", "fine", 0),
    ((6, 5, 8), 4, (1.0, 1.0, 1.6), 6000, "fp64", "ngp", "bulk", 0),
    ((7, 6, 5), 2, (0.7, 0.6, 0.5), 5000, "fp32n", "cic", "fine", 0),
    ((33, 17, 9), 4, (1.0, 0.5, 0.25), 70000, "fp32w", "cic", "fine", 1),
    ((12, 10, 8), 4, (1.2, 1.0, 0.8), 20000, "fp32k", "cic", "fine", 0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-r{c[1]}-n{c[3]}-{c[4]}-{c[5]}-{c[6]}-semi{c[7]}" for c in CASES])
def test_vof_parity(env, case):
    torch, cpl, oracle = env
    nb, r, box, n, prec, dep, src, semi = case
    precision = {"fp32w": cpl.COUPLE_FP32_WIDE, "fp32k": cpl.COUPLE_FP32_KAHAN, "fp32n": cpl.COUPLE_FP32_NAIVE, "fp64": cpl.COUPLE_FP64}[prec]
    w = W.small_workload(nb=nb, ratio=r, box=box, n=n, seed=400 + CASES.index(case),
                         precision="fp64" if prec == "fp64" else "fp32", deposit=dep)
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    alpha = W.fine_alpha(w)
    cfg = cfg_for(cpl, w, n, precision=precision, vel_source={"fine": 0, "bulk": 1}[src])
    cfg.vof, cfg.rho_f2, cfg.mu_f2, cfg.semi_implicit = 1, RHO2, MU2, semi
    print(f"case vof {case}", flush=True)
    g = run_gpu(cpl, torch, cfg, pos, vel, d, fine, alpha=alpha)
    o = oracle.step(pos, vel, d, fine, w.grid, rho_f=cfg.rho_f, mu_f=cfg.mu_f, rho_p=cfg.rho_p,
                    eps_min=cfg.eps_min, cic=dep == "cic", prec32=prec != "fp64", vel_source=src,
                    semi_implicit=bool(semi), alpha=alpha, rho2=RHO2, mu2=MU2)
    fp64 = prec == "fp64"
    errs = compare_step(g, o, n, nb, r, fp64=fp64, label=str(case), naive=prec == "fp32n", box=box)
    tol = TOL_FP64_FIELD if fp64 else (TOL_NAIVE if prec == "fp32n" else TOL_FP32_FIELD)
    ea = emax(g["bulk_alpha"].ravel(), o["alpha"], field_scale=1.0)
    assert ea <= tol, f"alpha e_max {ea:.3e}"
    # both fluids are present among the particles
    assert (o["alpha_p"] > 0.9).any() and (o["alpha_p"] < 0.1).any()
    print("vof e_max:", {k: f"{v:.2e}" for k, v in errs.items()}, f"alpha {ea:.2e}")


def test_vof_all_liquid_is_single_fluid_bitwise(env):
    """alpha = 1 everywhere: every output equals the single-fluid step's bit for bit."""
    torch, cpl, _ = env
    w = W.small_workload(nb=(10, 9, 7), ratio=4, box=(1.0, 0.9, 0.7), n=20000, seed=410, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    runs = []
    for vof in (0, 1):
        cfg = cfg_for(cpl, w, pos.shape[0], advect=1, dt=1e-4)
        cfg.vof = vof
        print(f"case vof all-liquid vof={vof}", flush=True)
        alpha = np.ones(cfg.nf[::-1], dtype=np.float32) if vof else None
        runs.append(run_gpu(cpl, torch, cfg, pos, vel, d, fine, alpha=alpha))
    a, b = runs
    for k in ("cell", "perm", "bulk_phi", "bulk_F", "bulk_U", "bulk_P", "bulk_G", "fine_eps", "fine_F", "drag",
              "beta", "pos_new", "vel_new"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert (b["bulk_alpha"] == 1.0).all()


def test_vof_needs_alpha(env):
    torch, cpl, _ = env
    w = W.small_workload(nb=(4, 4, 4), ratio=2, n=100, seed=411, precision="fp32")
    pos, d, vel = W.particles(w)
    cfg = cfg_for(cpl, w, 100)
    cfg.vof = 1
    dev = "cuda:0"
    c = cpl.Coupler(cfg)
    try:
        fine = [torch.zeros(cfg.nf[::-1], device=dev) for _ in range(4)]
        P = torch.from_numpy(pos.astype(np.float32)).to(dev)
        V = torch.from_numpy(vel.astype(np.float32)).to(dev)
        D = torch.from_numpy(d.astype(np.float32)).to(dev)
        with pytest.raises(cpl.CoupleError) as ei:
            c.step(P, V, D, fine)
        assert ei.value.code == cpl.COUPLE_EINVAL and "vof" in str(ei.value)
    finally:
        c.close()


def test_zero_particles_with_semi_implicit_and_two_fluid(env):
    """No particles, both options on: alpha is still restricted (against the
    oracle), K, KU and their prolongations are zero, every sum is zero."""
    torch, cpl, oracle = env
    w = W.small_workload(nb=(6, 5, 4), ratio=4, n=0, seed=3, precision="fp32")
    pos, d, vel = (np.zeros((0, 3), np.float32), np.zeros(0, np.float32), np.zeros((0, 3), np.float32))
    alpha = W.fine_alpha(w)
    cfg = cfg_for(cpl, w, 0)
    cfg.vof, cfg.rho_f2, cfg.mu_f2, cfg.semi_implicit = 1, RHO2, MU2, 1
    print("case zero particles semi + vof", flush=True)
    g = run_gpu(cpl, torch, cfg, pos, vel, d, W.fine_fields(w), alpha=alpha)
    a_ref = oracle.restrict(alpha, w.grid.nb, w.grid.ratio)
    assert emax(g["bulk_alpha"].ravel(), a_ref, field_scale=1.0) <= TOL_FP32_FIELD
    for k in ("bulk_K", "bulk_KU", "fine_K", "fine_KU", "bulk_phi", "bulk_F", "fine_F"):
        assert np.all(g[k] == 0), k
    for k in ("K_p", "K_b", "K_f"):
        assert g["diag_d"][k] == 0.0
    assert all(v == 0.0 for v in g["diag_d"]["KU_f"])

