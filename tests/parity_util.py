"""Helpers shared by the GPU parity tests: run one step through the C ABI and
compare it with the FP64 oracle.

Error metric (e_max) of a field g against the oracle o, element i:

    e_i = |g_i - o_i| / max(m_i, 1e-3 * S)

|.| is the Euclidean norm over the components of a vector element (a particle's
drag, a cell's U, G or F_fpi), the absolute value for scalars.  m_i is the size
of the element and S the size of the field's inputs, as the arithmetic sees them:
  * phi, drag, beta, fine eps: m_i = |o_i|, S = max_j m_j;
  * U, P (averages of fine values that may cancel): m_i = |o_i|, S = max of the
    average of the magnitudes |u_f|, |p_f| over the children;
  * G (differences of P): m_i = |o_i|, S = that pressure scale / min(h);
  * F_fpi (sums of drags that may cancel): m_i = S_i = the sum of the magnitudes
    of its terms M_c = (1/V_b) sum_p w_pc |F_p|;
  * prolonged F_fpi: m_i = max of M over the 27 bulk cells that feed the parent.
"""
import os

import numpy as np

# Tolerances of the parity contract.
TOL_FP32_FIELD = 1e-4     # e_max of every FP32 output field
TOL_FP64_FIELD = 1e-6     # every field of the FP64 mode (expect ~1e-12)
TOL_REDUCTION = 1e-6      # relative error of the FP64 global sums
# Naive (uncompensated) FP32 is the precision-study baseline, not the default
# path; its per-cell sums carry a few ulp more and its errors are reported.
TOL_NAIVE = 1e-3


def _norm(a):
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt((a ** 2).sum(axis=0)) if a.ndim == 2 else np.abs(a)


def emax(got, ref, mag=None, detail=False, field_scale=None):
    """e_max as defined in the module docstring.  Vector fields are [3, n]."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return (0.0, None) if detail else 0.0
    diff = _norm(got - ref).ravel()
    m = (_norm(ref) if mag is None else np.asarray(mag, dtype=np.float64)).ravel()
    S = m.max() if field_scale is None else max(float(field_scale), m.max())
    scale = np.maximum(m, 1e-3 * S)
    scale[scale == 0] = 1.0
    e = diff / scale
    i = int(np.nanargmax(e)) if np.isfinite(e).any() else 0
    val = float(np.nan_to_num(e, nan=np.inf).max())
    if detail:
        g2 = got.reshape(got.shape[0], -1)[:, i] if got.ndim == 2 else got.ravel()[i]
        r2 = ref.reshape(ref.shape[0], -1)[:, i] if ref.ndim == 2 else ref.ravel()[i]
        return val, dict(index=i, got=np.asarray(g2).tolist(), ref=np.asarray(r2).tolist(), scale=float(scale[i]))
    return val


def rms_rel(got, ref):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.sqrt(np.mean(ref ** 2)) or 1.0
    return float(np.sqrt(np.mean((got - ref) ** 2)) / den)


def neighbourhood_max(M, nb):
    """max over the 27 bulk cells around each cell (indices clamped)."""
    a = np.asarray(M, dtype=np.float64).reshape(nb[2], nb[1], nb[0])
    out = a.copy()
    for ax in range(3):
        lo = np.concatenate([a.take([0], axis=ax), a.take(range(a.shape[ax] - 1), axis=ax)], axis=ax)
        hi = np.concatenate([a.take(range(1, a.shape[ax]), axis=ax), a.take([a.shape[ax] - 1], axis=ax)], axis=ax)
        a = np.maximum(np.maximum(lo, hi), a)
    return a.ravel()


def fine_scale_from_bulk(Mb, nb, r, fine_index=None):
    """Bulk per-cell scale broadcast to the fine cells (or to sampled indices)."""
    Mb = np.asarray(Mb).reshape(nb[2], nb[1], nb[0])
    if fine_index is None:
        return np.repeat(np.repeat(np.repeat(Mb, r, 0), r, 1), r, 2).ravel()
    nf = [n * r for n in nb]
    f = np.asarray(fine_index, dtype=np.int64)
    i, j, k = f % nf[0], (f // nf[0]) % nf[1], f // (nf[0] * nf[1])
    return Mb[k // r, j // r, i // r]


def cfg_for(cpl, w, n, precision=None, deposit=None, vel_source=None, advect=None, dt=None):
    prec = precision if precision is not None else (cpl.COUPLE_FP64 if w.precision == "fp64" else cpl.COUPLE_FP32_WIDE)
    dep = deposit if deposit is not None else (cpl.COUPLE_CIC if w.deposit == "cic" else cpl.COUPLE_NGP)
    return cpl.Config(box=w.grid.box, nb=w.grid.nb, ratio=w.grid.ratio, rho_f=w.rho_f, mu_f=w.mu_f,
                      rho_p=w.rho_p, eps_min=w.eps_min, deposit=dep, precision=prec,
                      vel_source=cpl.COUPLE_VEL_FINE if vel_source is None else vel_source,
                      advect=int(w.advect if advect is None else advect), dt=w.dt if dt is None else dt,
                      max_particles=max(n, 1))


def to_dev(a, torch, dev, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def run_gpu(cpl, torch, cfg, pos, vel, diam, fine, uf_given=None, dev="cuda:0", alpha=None):
    """One step on the GPU; returns numpy copies of every output (+ advected state)."""
    dt = cfg.dtype
    P = to_dev(pos, torch, dev, dt)
    V = to_dev(vel, torch, dev, dt)
    D = to_dev(diam, torch, dev, dt)
    Fn = [to_dev(f, torch, dev, dt) for f in fine]
    UG = None if uf_given is None else to_dev(uf_given, torch, dev, dt)
    AL = None if alpha is None else to_dev(alpha, torch, dev, dt)
    c = cpl.Coupler(cfg)
    out = c.step(P, V, D, Fn, uf_given=UG, alpha=AL)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["diag_d"] = cpl.diag_dict(out["diag"])
    res["pos_new"] = P.cpu().numpy()
    res["vel_new"] = V.cpu().numpy()
    c.close()
    return res


def compare_step(g, o, n, nb, r, fp64, check_fine=True, fine_sample=None, label="", naive=False, box=(1.0, 1.0, 1.0),
                 fine_sample_index=None):
    """Assert parity of GPU outputs ``g`` with oracle outputs ``o``; returns errors.

    ``fine_sample`` indexes the GPU's fine outputs to match the oracle's sampled
    ones; ``fine_sample_index`` gives the fine cells those samples are (defaults
    to ``fine_sample``), for the error scale."""
    tol = TOL_FP64_FIELD if fp64 else (TOL_NAIVE if naive else TOL_FP32_FIELD)
    ncell = int(np.prod(nb))
    errs = {}
    np.testing.assert_array_equal(g["cell"], o["cell"], err_msg=label + " cell")
    np.testing.assert_array_equal(g["perm"], o["perm"], err_msg=label + " perm")
    np.testing.assert_array_equal(g["count"].ravel(), o["count"], err_msg=label + " count")
    np.testing.assert_array_equal(g["start"], o["start"], err_msg=label + " start")
    Mb = o["F_mag"]
    su = float(_norm(o["U_mag"]).max()) if ncell else 0.0
    sp = float(np.abs(o["P_mag"]).max()) if ncell else 0.0
    hmin = min(box[a] / nb[a] for a in range(3))
    fields = {
        "phi": (g["bulk_phi"].ravel(), o["phi"], None, None),
        "U": (g["bulk_U"].reshape(3, -1), o["U"], None, su),
        "P": (g["bulk_P"].ravel(), o["P"], None, sp),
        "G": (g["bulk_G"].reshape(3, -1), o["G"], None, sp / hmin),
        "F": (g["bulk_F"].reshape(3, -1), o["F"], Mb, None),
        "drag": (g["drag"].T, o["drag"].T, None, None),
        "beta": (g["beta"], o["beta"], None, None),
    }
    if o.get("pos_new") is not None and g.get("pos_new") is not None:
        # explicit Euler advection: the state after the step, per particle
        fields["pos_new"] = (np.asarray(g["pos_new"]).reshape(-1, 3).T, o["pos_new"].T, None, None)
        fields["vel_new"] = (np.asarray(g["vel_new"]).reshape(-1, 3).T, o["vel_new"].T, None, None)
    if check_fine:
        fidx = fine_sample if fine_sample_index is None else fine_sample_index
        Mf = fine_scale_from_bulk(neighbourhood_max(Mb, nb), nb, r, fidx)
        if fine_sample is None:
            fields["fine_eps"] = (g["fine_eps"].ravel(), o["fine_eps"], None, None)
            fields["fine_F"] = (g["fine_F"].reshape(3, -1), o["fine_F"], Mf, None)
        else:
            fields["fine_eps"] = (g["fine_eps"].ravel()[fine_sample], o["fine_eps"], None, None)
            fields["fine_F"] = (g["fine_F"].reshape(3, -1)[:, fine_sample], o["fine_F"], Mf, None)
    for name, (a, b, m, S) in fields.items():
        e, det = emax(a, b, m, detail=True, field_scale=S)
        errs[name] = e
        assert e <= tol, f"{label} {name}: e_max {e:.3e} > {tol}; worst {det}"
    d, od = g["diag_d"], o["diag"]
    rel = lambda x, y, s: abs(x - y) / max(abs(s), 1e-300)
    assert rel(d["V_tot"], od["V_tot"], od["V_tot"]) <= TOL_REDUCTION or n == 0
    assert rel(d["V_dep"], od["V_dep"], od["V_tot"]) <= TOL_REDUCTION or n == 0
    sabs = np.abs(o["drag"]).sum(axis=0) if n else np.ones(3)
    for a in range(3):
        s = max(sabs[a], 1e-300)
        assert abs(d["sum_Fp"][a] - od["sum_Fp"][a]) <= TOL_REDUCTION * s, label + " sum_Fp"
        assert abs(d["S_b"][a] - od["S_b"][a]) <= TOL_REDUCTION * s, label + " S_b"
        # equal and opposite, on the GPU's own numbers
        assert abs(d["S_b"][a] + d["sum_Fp"][a]) <= TOL_REDUCTION * s, label + " S_b = -sum F_p"
        if check_fine:
            assert abs(d["S_f"][a] - d["S_b"][a]) <= TOL_REDUCTION * s, label + " S_f = S_b"
    assert d["n_outside"] == od["n_outside"], label + " n_outside"
    assert abs(d["n_clamped"] - od["n_clamped"]) <= max(2, 1e-5 * n), label + " n_clamped"
    if ncell:
        assert abs(d["max_phi"] - od["max_phi"]) <= TOL_REDUCTION * max(od["max_phi"], 1e-300) + 1e-7
    if check_fine and fine_sample is None and "E_f" in od:
        assert rel(d["E_f"], od["E_f"], od["E_f"]) <= TOL_REDUCTION
    return errs


def raw_step(cpl, h, inputs, outputs, stream=None):
    """Call the C entry point directly, without the binding's argument checks
    (to test the library's own checks); returns the status code."""
    import ctypes as C
    i = cpl._Inputs()
    i.n = int(inputs["n"])
    for k, _ in cpl._Inputs._fields_:
        if k not in ("n", "step"):
            t = inputs.get(k)
            setattr(i, k, None if t is None else t.data_ptr())
    o = cpl._Outputs()
    for k, _ in cpl._Outputs._fields_:
        t = outputs.get(k)
        setattr(o, k, None if t is None else t.data_ptr())
    return cpl._lib.couple_step(h, C.byref(i), C.byref(o), cpl._stream(stream))


def results_dir():
    """Where GPU tests write their reports (JSON): $COUPLE_RESULTS_DIR, else
    results/ at the repository root."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return os.environ.get("COUPLE_RESULTS_DIR") or os.path.join(root, "results")
