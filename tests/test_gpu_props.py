"""GPU parity on tiny random configurations drawn by hypothesis (derandomized,
so every run draws the same cases): grid shape, ratio, box, particle count
(including none), precision, weights, velocity source, and the semi-implicit
split and two-fluid drag options.  Each case is compared with the FP64 oracle
as in test_gpu_parity (bit-exact integers, e_max bounds, FP64 sums)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import workload as W
from parity_util import TOL_FP32_FIELD, TOL_FP64_FIELD, TOL_NAIVE, cfg_for, compare_step, emax, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


cases = st.fixed_dictionaries({
    "nb": st.tuples(st.integers(1, 9), st.integers(1, 9), st.integers(1, 9)),
    "ratio": st.sampled_from([1, 2, 4]),
    "box": st.tuples(st.floats(0.1, 2.0), st.floats(0.1, 2.0), st.floats(0.1, 2.0)),
    "n": st.integers(0, 5000),
    "prec": st.sampled_from(["fp64", "fp32w", "fp32k", "fp32n"]),
    "cic": st.booleans(),
    "src": st.sampled_from(["fine", "bulk"]),
    "semi": st.booleans(),
    "vof": st.booleans(),
    "seed": st.integers(0, 100_000),
})


@settings(max_examples=25, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(c=cases)
def test_random_tiny_configurations(env, c):
    torch, cpl, oracle = env
    fp64 = c["prec"] == "fp64"
    # at most a mean solid fraction of 0.3 (spheres of mean diameter 0.02): a
    # box packed towards phi = 1 leaves eps = 1 - phi with a few FP32 digits
    vol = c["box"][0] * c["box"][1] * c["box"][2]
    c = {**c, "n": min(c["n"], int(0.3 * vol / (np.pi / 6 * 0.02 ** 3)))}
    w = W.small_workload(nb=c["nb"], ratio=c["ratio"], box=c["box"], n=c["n"], seed=c["seed"],
                         precision="fp64" if fp64 else "fp32", deposit="cic" if c["cic"] else "ngp")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    alpha = W.fine_alpha(w) if c["vof"] else None
    precision = {"fp32w": cpl.COUPLE_FP32_WIDE, "fp32k": cpl.COUPLE_FP32_KAHAN, "fp32n": cpl.COUPLE_FP32_NAIVE, "fp64": cpl.COUPLE_FP64}[c["prec"]]
    cfg = cfg_for(cpl, w, c["n"], precision=precision, vel_source={"fine": 0, "bulk": 1}[c["src"]])
    cfg.semi_implicit, cfg.vof = int(c["semi"]), int(c["vof"])
    print(f"case props {c}", flush=True)
    g = run_gpu(cpl, torch, cfg, pos, vel, d, fine, alpha=alpha)
    o = oracle.step(pos, vel, d, fine, w.grid, rho_f=cfg.rho_f, mu_f=cfg.mu_f, rho_p=cfg.rho_p, eps_min=cfg.eps_min,
                    cic=c["cic"], prec32=not fp64, vel_source=c["src"], semi_implicit=c["semi"], alpha=alpha,
                    rho2=cfg.rho_f2, mu2=cfg.mu_f2)
    compare_step(g, o, c["n"], w.grid.nb, w.grid.ratio, fp64=fp64, naive=c["prec"] == "fp32n", box=w.grid.box,
                 label=str(c))
    tol = TOL_FP64_FIELD if fp64 else (TOL_NAIVE if c["prec"] == "fp32n" else TOL_FP32_FIELD)
    if c["semi"] and c["n"] > 0:
        nc = int(np.prod(w.grid.nb))
        assert emax(g["bulk_K"].ravel(), o["K"]) <= tol
        assert emax(g["bulk_KU"].reshape(3, nc), o["KU"], o["KU_mag"]) <= tol
    if c["vof"]:
        assert emax(g["bulk_alpha"].ravel(), o["alpha"], field_scale=1.0) <= tol
