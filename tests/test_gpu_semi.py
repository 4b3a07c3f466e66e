"""GPU parity of the semi-implicit split of the momentum source (the drag term of
Eq. UFP treated semi-implicitly, Sec. 2.5): K_c = (1/V_b) sum_p w_pc beta_p and
KU_c = (1/V_b) sum_p w_pc beta_p u_p on the bulk grid, both prolonged to the fine
grid, and their FP64 sums, against the FP64 oracle through the C ABI.

Error metric as in parity_util: K (a sum of positive terms) relative to itself;
KU relative to the sum of its terms' magnitudes (1/V_b) sum_p w_pc beta_p |u_p|;
the prolonged fields relative to the largest bulk scale of the 27 cells that
feed the parent cell.
"""
import numpy as np
import pytest

import workload as W
from parity_util import (TOL_FP32_FIELD, TOL_FP64_FIELD, TOL_NAIVE, TOL_REDUCTION, cfg_for, compare_step, emax,
                         fine_scale_from_bulk, neighbourhood_max, run_gpu)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


CASES = [
    # (nb, ratio, box, n, precision, deposit, vel_source, advect)
    ((5, 3, 4), 4, (1.0, 0.75, 1.25), 777, "fp32w", "cic", "fine", 0),
    ((6, 5, 4), 4, (1.0, 1.0, 1.0), 4000, "fp64", "ngp", "bulk", 0),
    ((7, 6, 5), 2, (0.7, 0.6, 0.5), 5000, "fp32n", "cic", "fine", 0),
    ((9, 4, 3), 1, (0.9, 0.4, 0.3), 4097, "fp32w", "ngp", "fine", 1),
    ((33, 17, 9), 4, (1.0, 0.5, 0.25), 70000, "fp32w", "cic", "fine", 1),
    ((12, 9, 7), 4, (1.2, 0.9, 0.7), 30000, "fp32k", "cic", "fine", 1),
    ((6, 5, 4), 2, (1.0, 1.0, 1.0), 4000, "fp32k", "ngp", "bulk", 0),
]


def _semi_errors(g, o, nb, r, tol, label):
    nc = int(np.prod(nb))
    K, KU = o["K"], o["KU"]
    Mk = np.abs(K)
    Mku = o["KU_mag"]
    fields = {
        "K": (g["bulk_K"].ravel(), K, None),
        "KU": (g["bulk_KU"].reshape(3, nc), KU, Mku),
        "fine_K": (g["fine_K"].ravel(), o["fine_K"], fine_scale_from_bulk(neighbourhood_max(Mk, nb), nb, r)),
        "fine_KU": (g["fine_KU"].reshape(3, -1), o["fine_KU"],
                    fine_scale_from_bulk(neighbourhood_max(Mku, nb), nb, r)),
    }
    errs = {}
    for name, (a, b, m) in fields.items():
        e, det = emax(a, b, m, detail=True)
        errs[name] = e
        assert e <= tol, f"{label} {name}: e_max {e:.3e} > {tol}; worst {det}"
    return errs


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-r{c[1]}-n{c[3]}-{c[4]}-{c[5]}-{c[6]}-adv{c[7]}" for c in CASES])
def test_semi_parity(env, case):
    torch, cpl, oracle = env
    nb, r, box, n, prec, dep, src, adv = case
    precision = {"fp32w": cpl.COUPLE_FP32_WIDE, "fp32k": cpl.COUPLE_FP32_KAHAN, "fp32n": cpl.COUPLE_FP32_NAIVE, "fp64": cpl.COUPLE_FP64}[prec]
    w = W.small_workload(nb=nb, ratio=r, box=box, n=n, seed=300 + CASES.index(case),
                         precision="fp64" if prec == "fp64" else "fp32", deposit=dep)
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    cfg = cfg_for(cpl, w, n, precision=precision, vel_source={"fine": 0, "bulk": 1}[src], advect=adv,
                  dt=1e-4 if adv else 0.0)
    cfg.semi_implicit = 1
    print(f"case semi {case}", flush=True)
    g = run_gpu(cpl, torch, cfg, pos, vel, d, fine)
    o = oracle.step(pos, vel, d, fine, w.grid, rho_f=cfg.rho_f, mu_f=cfg.mu_f, rho_p=cfg.rho_p,
                    eps_min=cfg.eps_min, cic=dep == "cic", prec32=prec != "fp64", vel_source=src,
                    advect_dt=cfg.dt if adv else None, semi_implicit=True)
    fp64 = prec == "fp64"
    compare_step(g, o, n, nb, r, fp64=fp64, label=str(case), naive=prec == "fp32n", box=box)
    tol = TOL_FP64_FIELD if fp64 else (TOL_NAIVE if prec == "fp32n" else TOL_FP32_FIELD)
    errs = _semi_errors(g, o, nb, r, tol, str(case))
    print("semi e_max:", {k: f"{v:.2e}" for k, v in errs.items()})
    d_, od = g["diag_d"], o["diag"]
    kp = od["K_p"]
    assert abs(d_["K_p"] - kp) <= TOL_REDUCTION * kp
    assert abs(d_["K_b"] - d_["K_p"]) <= TOL_REDUCTION * kp       # deposition conserves
    assert abs(d_["K_f"] - d_["K_b"]) <= TOL_REDUCTION * kp       # prolongation conserves
    bu = np.abs(o["beta"][:, None] * vel).sum(axis=0)
    for a in range(3):
        assert abs(d_["KU_p"][a] - od["KU_p"][a]) <= TOL_REDUCTION * bu[a]
        assert abs(d_["KU_b"][a] - d_["KU_p"][a]) <= TOL_REDUCTION * bu[a]
        assert abs(d_["KU_f"][a] - d_["KU_b"][a]) <= TOL_REDUCTION * bu[a]


def test_semi_split_reproduces_source_in_uniform_flow(env):
    """Given the same fluid velocity U0 at every particle, the GPU's own outputs
    satisfy F_fpi = -K U0 + KU (up to FP32 rounding of the sums)."""
    torch, cpl, _ = env
    w = W.small_workload(nb=(12, 10, 8), ratio=4, box=(1.2, 1.0, 0.8), n=30000, seed=310, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    U0 = np.array([0.25, -0.5, 0.125])
    cfg = cfg_for(cpl, w, pos.shape[0], vel_source=cpl.COUPLE_VEL_GIVEN)
    cfg.semi_implicit = 1
    print("case semi uniform flow", flush=True)
    g = run_gpu(cpl, torch, cfg, pos, vel, d, fine, uf_given=np.broadcast_to(U0, pos.shape).astype(np.float32))
    nc = int(np.prod(w.grid.nb))
    F, K, KU = g["bulk_F"].reshape(3, nc).astype(np.float64), g["bulk_K"].ravel().astype(np.float64), \
        g["bulk_KU"].reshape(3, nc).astype(np.float64)
    pred = -K[None, :] * U0[:, None] + KU
    scale = np.abs(K)[None, :] * np.abs(U0)[:, None] + np.abs(KU)
    e = emax(F, pred, np.sqrt((scale ** 2).sum(axis=0)))
    print(f"uniform-flow split e_max {e:.2e}")
    assert e <= TOL_FP32_FIELD


def test_semi_leaves_plain_outputs_unchanged(env):
    """Turning the split on changes no other output, bit for bit (advection on)."""
    torch, cpl, _ = env
    w = W.small_workload(nb=(10, 9, 7), ratio=4, box=(1.0, 0.9, 0.7), n=20000, seed=311, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    runs = []
    for semi in (0, 1):
        cfg = cfg_for(cpl, w, pos.shape[0], advect=1, dt=1e-4)
        cfg.semi_implicit = semi
        print(f"case semi plain-unchanged semi={semi}", flush=True)
        runs.append(run_gpu(cpl, torch, cfg, pos, vel, d, fine))
    a, b = runs
    for k in ("cell", "perm", "count", "start", "bulk_phi", "bulk_F", "bulk_U", "bulk_P", "bulk_G", "fine_eps",
              "fine_F", "drag", "beta", "pos_new", "vel_new"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for k in ("V_tot", "V_dep", "sum_Fp", "S_b", "S_f", "E_f", "n_clamped", "n_outside", "max_phi"):
        assert a["diag_d"][k] == b["diag_d"][k], k
    assert a["diag_d"]["K_p"] == 0.0 and b["diag_d"]["K_p"] > 0.0


def test_semi_needs_its_outputs(env):
    torch, cpl, _ = env
    w = W.small_workload(nb=(4, 4, 4), ratio=2, n=100, seed=312, precision="fp32")
    pos, d, vel = W.particles(w)
    cfg = cfg_for(cpl, w, 100)
    cfg.semi_implicit = 1
    dev = "cuda:0"
    c = cpl.Coupler(cfg)
    try:
        out = cpl.alloc_outputs(cfg, 100, device=dev)
        out["fine_KU"] = None
        fine = [torch.zeros(cfg.nf[::-1], device=dev) for _ in range(4)]
        P = torch.from_numpy(pos.astype(np.float32)).to(dev)
        V = torch.from_numpy(vel.astype(np.float32)).to(dev)
        D = torch.from_numpy(d.astype(np.float32)).to(dev)
        with pytest.raises(cpl.CoupleError) as ei:
            c.step(P, V, D, fine, out=out)
        assert ei.value.code == cpl.COUPLE_EINVAL and "semi_implicit" in str(ei.value)
    finally:
        c.close()
