"""The binding's argument checks (CPU): every tensor handed to the library is
checked for device, dtype, size, contiguity and alignment against the
configuration before its address is passed on, so that a wrong argument raises
instead of sending the kernels out of bounds."""
import pytest
import torch

cpl = pytest.importorskip("paper_1807_11834_amd")


def _cfg(**kw):
    return cpl.Config(**{"nb": (4, 3, 2), "ratio": 2, "max_particles": 10, **kw})


def _args(cfg, n, dtype=None):
    dt = dtype or cfg.dtype
    nb, nf = cfg.n_bulk, cfg.n_fine
    z = lambda *s, d=dt: torch.zeros(*s, dtype=d)
    inputs = {"n": n, "pos": z(n, 3), "vel": z(n, 3), "diam": z(n), "fine_u": z(nf), "fine_v": z(nf),
              "fine_w": z(nf), "fine_p": z(nf)}
    outputs = {"drag": z(n, 3), "beta": z(n), "cell": z(n, d=torch.int32), "perm": z(n, d=torch.int32),
               "count": z(nb, d=torch.int32), "start": z(nb + 1, d=torch.int32), "bulk_phi": z(nb),
               "bulk_F": z(3, nb), "bulk_U": z(3, nb), "bulk_P": z(nb), "bulk_G": z(3, nb), "fine_eps": z(nf),
               "fine_F": z(3, nf), "diag": z(cpl.DIAG_LEN, d=torch.float64)}
    return inputs, outputs


def test_valid_arguments_pass():
    for prec in (cpl.COUPLE_FP32_WIDE, cpl.COUPLE_FP64):
        cfg = _cfg(precision=prec)
        i, o = _args(cfg, 7)
        cpl.validate_step(cfg, i, o, require_gpu=False)
        i, o = _args(cfg, 0)
        for k in ("pos", "vel", "diam"):
            i[k] = None
        for k in ("drag", "cell", "perm"):
            o[k] = None
        cpl.validate_step(cfg, i, o, require_gpu=False)   # no particles: particle arrays may be NULL


def test_cpu_tensors_are_rejected():
    cfg = _cfg()
    i, o = _args(cfg, 3)
    with pytest.raises(ValueError, match="must be on a GPU"):
        cpl.validate_step(cfg, i, o)


@pytest.mark.parametrize("what", ["dtype", "size", "strided", "offset", "int_dtype", "diag", "capacity", "missing",
                                  "not_tensor"])
def test_bad_arguments_raise(what):
    cfg = _cfg()
    i, o = _args(cfg, 5)
    code = cpl.COUPLE_EINVAL
    if what == "dtype":
        i["pos"] = i["pos"].double()                  # FP64 data on an FP32 handle
    elif what == "size":
        i["fine_u"] = torch.zeros(cfg.n_fine - 1)      # one fine cell short
    elif what == "strided":
        o["drag"] = torch.zeros(3, 5).t()              # transposed view
    elif what == "offset":
        i["diam"] = torch.zeros(6)[1:]                 # a view starting 4 bytes in
    elif what == "int_dtype":
        o["perm"] = torch.zeros(5, dtype=torch.int64)
    elif what == "diag":
        o["diag"] = torch.zeros(cpl.DIAG_LEN)          # FP32 diagnostics
    elif what == "capacity":
        i, o = _args(cfg, 11)
        code = cpl.COUPLE_ECAPACITY
    elif what == "missing":
        o["bulk_G"] = None
    else:
        i["vel"] = [0.0] * 15
    with pytest.raises(cpl.ArgumentError) as ei:
        cpl.validate_step(cfg, i, o, require_gpu=False)
    assert isinstance(ei.value, ValueError) and ei.value.code == code


def test_mode_dependent_arguments():
    cfg = _cfg(semi_implicit=1, vof=1, vel_source=cpl.COUPLE_VEL_GIVEN)
    i, o = _args(cfg, 4)
    with pytest.raises(ValueError, match="uf_given: required with vel_source GIVEN"):
        cpl.validate_step(cfg, i, o, require_gpu=False)
    i["uf_given"] = torch.zeros(4, 3)
    with pytest.raises(ValueError, match="fine_alpha: required with vof = 1"):
        cpl.validate_step(cfg, i, o, require_gpu=False)
    i["fine_alpha"] = torch.zeros(cfg.n_fine)
    with pytest.raises(ValueError, match="bulk_K: required with semi_implicit = 1"):
        cpl.validate_step(cfg, i, o, require_gpu=False)
    o.update(bulk_K=torch.zeros(cfg.n_bulk), bulk_KU=torch.zeros(3 * cfg.n_bulk), fine_K=torch.zeros(cfg.n_fine),
             fine_KU=torch.zeros(3 * cfg.n_fine))
    with pytest.raises(ValueError, match="bulk_alpha"):
        cpl.validate_step(cfg, i, o, require_gpu=False)
    o["bulk_alpha"] = torch.zeros(cfg.n_bulk)
    cpl.validate_step(cfg, i, o, require_gpu=False)


def test_check_tensor_device_mismatch():
    t = torch.zeros(4)
    with pytest.raises(ValueError, match="other arguments"):
        cpl.check_tensor("x", t, torch.float32, 4, device=torch.device("meta"), require_gpu=False)
    cpl.check_tensor("x", None, torch.float32, 4, optional=True)


def test_step_needs_a_live_handle():
    import ctypes as C
    cfg = _cfg()
    i, o = _args(cfg, 1)
    with pytest.raises(ValueError, match="live handle"):
        cpl.couple_step(C.c_void_p(12345), i, o)
