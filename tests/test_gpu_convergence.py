"""Grid convergence of the fine-grid lookup on the GPU: the fluid velocity the
step uses at the particles (trilinear on the fine cell centres) against the
analytic Taylor-Green field.  Trilinear interpolation of a smooth field is
second order, so halving the fine spacing divides the error by about four; the
error also stays below the tensor-product bound (3/8) k^2 h_f^2 A (reading of
the fine fields as point values at cell centres)."""
import math

import numpy as np
import pytest

import workload as W
from parity_util import cfg_for, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_11834_amd as cpl
    return torch, cpl


def test_fine_lookup_is_second_order(env):
    torch, cpl = env
    errs = []
    for nb in ((4, 4, 4), (8, 8, 8), (16, 16, 16)):
        w = W.small_workload(nb=nb, ratio=4, box=(1.0, 1.0, 1.0), n=20000, seed=600, precision="fp64")
        pos, d, vel = W.particles(w)
        cfg = cfg_for(cpl, w, pos.shape[0])
        print(f"case convergence nb={nb}", flush=True)
        dev = "cuda:0"
        c = cpl.Coupler(cfg)
        to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        out = c.step(to(pos), to(vel), to(d), [to(f) for f in W.fine_fields(w)], uf=True)
        torch.cuda.synchronize()
        uf = out["uf"].cpu().numpy()
        c.close()
        u, v, ww, _ = W.fluid_analytic(w, pos[:, 0], pos[:, 1], pos[:, 2])
        # particles at least one fine cell from the walls (the clamped lookup is
        # first order there)
        hf = 1.0 / (nb[0] * 4)
        inner = np.all((pos > hf) & (pos < 1.0 - hf), axis=1)
        e = np.abs(np.stack([u, v, ww], axis=1)[inner] - uf[inner]).max()
        bound = 3.0 / 8.0 * (2 * math.pi) ** 2 * hf ** 2 * 1.0 * 1.05
        print(f"h_f = {hf:.4g}: max error {e:.3e}, bound {bound:.3e}")
        assert e <= bound
        errs.append(e)
    for a, b in zip(errs[:-1], errs[1:]):
        assert 3.0 <= a / b <= 5.0, errs
