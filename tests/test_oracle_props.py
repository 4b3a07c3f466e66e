"""Property tests of the oracle on tiny random configurations (hypothesis).

Invariants that hold for every grid, ratio, weighting and particle set, checked
on configurations hypothesis draws (derandomized, so the suite is repeatable):
  * deposited volume equals the particle volume (Table 1 porosity definition);
  * the momentum source is equal and opposite to the drag (Eq. UFP, F_fpi);
  * the conservative prolongation keeps the source's and the porosity's sums
    and restricting it gives the bulk field back (R o P = I);
  * the semi-implicit fields keep the particle sums of beta and beta u_p;
  * the non-nested transfer keeps constants and the integral.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import workload as W

SETTINGS = settings(max_examples=30, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])

configs = st.fixed_dictionaries({
    "nb": st.tuples(st.integers(1, 6), st.integers(1, 6), st.integers(1, 6)),
    "ratio": st.sampled_from([1, 2, 4]),
    "n": st.integers(0, 400),
    "cic": st.booleans(),
    "seed": st.integers(0, 10_000),
    "box": st.tuples(st.floats(0.2, 2.0), st.floats(0.2, 2.0), st.floats(0.2, 2.0)),
})


@SETTINGS
@given(configs)
def test_step_invariants(orc, c):
    w = W.small_workload(nb=c["nb"], ratio=c["ratio"], box=c["box"], n=c["n"], seed=c["seed"], precision="fp64",
                         deposit="cic" if c["cic"] else "ngp")
    pos, d, vel = W.particles(w)
    o = orc.step(pos, vel, d, W.fine_fields(w), w.grid, cic=c["cic"], prec32=False, semi_implicit=True)
    dg = o["diag"]
    vt = max(dg["V_tot"], 1e-300)
    assert abs(dg["V_dep"] - dg["V_tot"]) <= 1e-12 * vt
    sabs = np.abs(o["drag"]).sum(axis=0) + 1e-300
    for a in range(3):
        assert abs(dg["S_b"][a] + dg["sum_Fp"][a]) <= 1e-12 * sabs[a]
        assert abs(dg["S_f"][a] - dg["S_b"][a]) <= 1e-11 * sabs[a]
    vol = float(np.prod(c["box"]))
    assert abs(dg["E_f"] - (vol - dg["V_dep"])) <= 1e-12 * vol
    kp = max(dg["K_p"], 1e-300)
    assert abs(dg["K_b"] - dg["K_p"]) <= 1e-12 * kp and abs(dg["K_f"] - dg["K_b"]) <= 1e-11 * kp
    bu = np.abs(o["beta"][:, None] * vel).sum(axis=0) + 1e-300
    for a in range(3):
        assert abs(dg["KU_b"][a] - dg["KU_p"][a]) <= 1e-12 * bu[a]
    # R o P = I for the prolonged porosity
    nb, r = w.grid.nb, w.grid.ratio
    np.testing.assert_allclose(orc.restrict(o["fine_eps"], nb, r), 1.0 - o["phi"], rtol=0, atol=1e-12)
    assert (o["count"] >= 0).all() and o["count"].sum() == c["n"]


nodes = st.lists(st.floats(0.05, 1.0), min_size=1, max_size=7)


@SETTINGS
@given(nodes, nodes, nodes, nodes, st.integers(0, 1000))
def test_remap_constants_and_integral(orc, sx, sy, dx, dy, seed):
    """Random rectilinear sender / receiver spacings along x and y (z one cell)."""
    def grid(widths, L=1.0):
        x = np.concatenate([[0.0], np.cumsum(widths)])
        x = x / x[-1] * L
        x[-1] = L
        return x
    S = [grid(sx), grid(sy), np.array([0.0, 0.5])]
    D = [grid(dx), grid(dy), np.array([0.0, 0.5])]
    ns = [len(a) - 1 for a in S]
    rng = np.random.default_rng(seed)
    s = rng.normal(size=(ns[2], ns[1], ns[0]))
    t = orc.remap(s, S, D)
    vs = np.diff(S[2])[:, None, None] * np.diff(S[1])[None, :, None] * np.diff(S[0])[None, None, :]
    vd = np.diff(D[2])[:, None, None] * np.diff(D[1])[None, :, None] * np.diff(D[0])[None, None, :]
    assert abs((t * vd).sum() - (s * vs).sum()) <= 1e-13 * (np.abs(s) * vs).sum() + 1e-300
    np.testing.assert_allclose(orc.remap(np.full_like(s, -2.5), S, D), -2.5, rtol=1e-14)
