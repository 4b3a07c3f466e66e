"""Python binding of the MI355X dual-grid coupling library (``libcouple.so``).

Argument marshalling only: every stage of a coupling step runs in the HIP
kernels behind the C ABI declared in ``include/couple.h``.  PyTorch provides the
device memory (tensors are passed as ``data_ptr()``) and the stream.  There is no
CPU fallback: importing this package without the built library raises.

The functions mirror the C entry points::

    h = couple_init(Config(...))
    couple_step(h, inputs, outputs, stream=None)
    couple_free(h)
    couple_last_error(h)

and those of the learned velocity surrogate (``include/couple_mlp.h``):
``couple_mlp_init / _free / _set_params / _set_norm / _fit_norm / _get_state /
_set_state / _forward / _grads / _adam / _train_step / _features`` and
``couple_set_mlp``.

``Coupler`` wraps a handle with output allocation, ``Mlp`` a network.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcouple.so")

# ---- constants (include/couple.h) -------------------------------------------
COUPLE_OK, COUPLE_EINVAL, COUPLE_ENOMEM, COUPLE_EHIP, COUPLE_ECAPACITY, COUPLE_ESTATE = 0, -1, -2, -3, -4, -6
COUPLE_NGP, COUPLE_CIC = 0, 1
COUPLE_FP64, COUPLE_FP32_WIDE, COUPLE_FP32_NAIVE, COUPLE_FP32_KAHAN = 0, 1, 2, 3
COUPLE_VEL_FINE, COUPLE_VEL_BULK, COUPLE_VEL_GIVEN, COUPLE_VEL_MLP = 0, 1, 2, 3
COUPLE_EXCHANGE_DISTRIBUTED, COUPLE_EXCHANGE_GATHER_SCATTER = 0, 1
COUPLE_HBMREF_READ, COUPLE_HBMREF_WRITE, COUPLE_HBMREF_COPY = 0, 1, 2
DIAG = {"V_tot": 0, "V_dep": 1, "sum_Fp": 2, "S_b": 5, "S_f": 8, "E_f": 11, "n_clamped": 12,
        "n_outside": 13, "max_phi": 14, "n_fallback": 15, "mlp_err2": 16, "mlp_ref2": 17, "mlp_nsamp": 18,
        "K_p": 19, "KU_p": 20, "K_b": 23, "KU_b": 24, "K_f": 27, "KU_f": 28}
DIAG_LEN = 31
MLP_NFEAT = 193
MLP_NPARAM = 58243


class CoupleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class ArgumentError(CoupleError, ValueError):
    """An argument rejected by the binding's checks before the library is
    called (the code is the one the library would return, where it checks)."""

    def __init__(self, msg, code=COUPLE_EINVAL):
        super().__init__(code, msg)


class _Config(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("nb", C.c_int32 * 3), ("ratio", C.c_int32),
                ("rho_f", C.c_double), ("mu_f", C.c_double), ("rho_p", C.c_double), ("eps_min", C.c_double),
                ("phi_fp64", C.c_double), ("deposit", C.c_int32), ("precision", C.c_int32),
                ("vel_source", C.c_int32), ("advect", C.c_int32), ("dt", C.c_double),
                ("max_particles", C.c_int64), ("mlp_tol", C.c_double), ("mlp_period", C.c_int32),
                ("semi_implicit", C.c_int32), ("vof", C.c_int32), ("rho_f2", C.c_double), ("mu_f2", C.c_double)]


class _Inputs(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.c_void_p), ("vel", C.c_void_p), ("diam", C.c_void_p),
                ("fine_u", C.c_void_p), ("fine_v", C.c_void_p), ("fine_w", C.c_void_p), ("fine_p", C.c_void_p),
                ("uf_given", C.c_void_p), ("step", C.c_int64), ("fine_alpha", C.c_void_p)]


class _Outputs(C.Structure):
    _fields_ = [("drag", C.c_void_p), ("beta", C.c_void_p), ("cell", C.c_void_p), ("perm", C.c_void_p),
                ("count", C.c_void_p), ("start", C.c_void_p), ("bulk_phi", C.c_void_p), ("bulk_F", C.c_void_p),
                ("bulk_U", C.c_void_p), ("bulk_P", C.c_void_p), ("bulk_G", C.c_void_p),
                ("fine_eps", C.c_void_p), ("fine_F", C.c_void_p), ("diag", C.c_void_p), ("uf", C.c_void_p),
                ("bulk_K", C.c_void_p), ("bulk_KU", C.c_void_p), ("fine_K", C.c_void_p), ("fine_KU", C.c_void_p),
                ("bulk_alpha", C.c_void_p)]


class _MlpConfig(C.Structure):
    _fields_ = [("max_batch", C.c_int64), ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


class _KernelStat(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_int64), ("total_ms", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(there is no CPU fallback for the coupling step)")
    L = C.CDLL(LIB_PATH)
    L.couple_init.argtypes = [C.POINTER(_Config), C.POINTER(C.c_void_p)]
    L.couple_init.restype = C.c_int
    L.couple_step.argtypes = [C.c_void_p, C.POINTER(_Inputs), C.POINTER(_Outputs), C.c_void_p]
    L.couple_step.restype = C.c_int
    L.couple_free.argtypes = [C.c_void_p]
    L.couple_free.restype = C.c_int
    L.couple_last_error.argtypes = [C.c_void_p]
    L.couple_last_error.restype = C.c_char_p
    L.couple_step_noalloc.argtypes = [C.POINTER(_Config), C.POINTER(_Inputs), C.POINTER(_Outputs), C.c_void_p]
    L.couple_step_noalloc.restype = C.c_int
    L.couple_timing_begin.argtypes = [C.c_void_p, C.c_int32]
    L.couple_timing_begin.restype = C.c_int
    L.couple_timing_end.argtypes = [C.c_void_p, C.POINTER(_KernelStat), C.c_int32, C.POINTER(C.c_int32)]
    L.couple_timing_end.restype = C.c_int
    P, I64, I = C.c_void_p, C.c_int64, C.c_int
    sigs = {
        "couple_mlp_init": [C.POINTER(_MlpConfig), C.POINTER(C.c_void_p)],
        "couple_mlp_free": [P],
        "couple_mlp_set_params": [P, P],
        "couple_mlp_set_norm": [P, P, P, P],
        "couple_mlp_fit_norm": [P, P, P, I64, P],
        "couple_mlp_get_state": [P, P, P, P, P, P, P, P],
        "couple_mlp_set_state": [P, P, P, P, I64, P, P, P],
        "couple_mlp_forward": [P, P, I64, P, P],
        "couple_mlp_grads": [P, P, P, I64, P, I64, P, P, P],
        "couple_mlp_adam": [P, P, P],
        "couple_mlp_train_step": [P, P, P, I64, P, I64, P, P],
        "couple_mlp_features": [C.POINTER(_Config), I64, P, P, P, P, P, P, P, I64, P, P, P, P],
        "couple_set_mlp": [P, P],
        "couple_remap_init": [P, P, P, P, C.c_int32, C.POINTER(C.c_void_p)],
        "couple_remap_apply": [P, P, P, C.c_int32, P],
        "couple_remap_info": [P, P, P],
        "couple_remap_free": [P],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I
    for name, args in {"couple_boxmap_init": [I64, P, I64, P, C.c_int32, C.POINTER(C.c_void_p)],
                       "couple_boxmap_apply": [P, P, P, C.c_int32, P],
                       "couple_boxmap_info": [P, P, P], "couple_boxmap_free": [P]}.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I
    L.couple_boxmap_last_error.argtypes = [P]
    L.couple_boxmap_last_error.restype = C.c_char_p
    for name, args in {"couple_part_init": [C.POINTER(_Config), C.c_int32, C.POINTER(C.c_void_p)],
                       "couple_part_step": [P, C.POINTER(_Inputs), C.POINTER(_Outputs), C.c_int32, P],
                       "couple_part_comm_matrix": [P, P], "couple_part_free": [P]}.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I
    L.couple_part_last_error.argtypes = [P]
    L.couple_part_last_error.restype = C.c_char_p
    L.couple_remap_last_error.argtypes = [P]
    L.couple_remap_last_error.restype = C.c_char_p
    L.couple_mlp_last_error.argtypes = [P]
    L.couple_mlp_last_error.restype = C.c_char_p
    L.couple_hbmref.argtypes = [I, P, P, I64, C.c_float, P]
    L.couple_hbmref.restype = I
    return L


_lib = _load()


@dataclass
class Config:
    """Mirror of ``couple_config``."""
    box: tuple = (1.0, 1.0, 1.0)
    nb: tuple = (8, 8, 8)
    ratio: int = 4
    rho_f: float = 1000.0
    mu_f: float = 1.0e-3
    rho_p: float = 2500.0
    eps_min: float = 0.3
    phi_fp64: float = 0.5
    deposit: int = COUPLE_CIC
    precision: int = COUPLE_FP32_WIDE
    vel_source: int = COUPLE_VEL_FINE
    advect: int = 0
    dt: float = 0.0
    max_particles: int = 0
    mlp_tol: float = 1.0e-3
    mlp_period: int = 100
    semi_implicit: int = 0
    vof: int = 0
    rho_f2: float = 1.2
    mu_f2: float = 1.8e-5

    def to_c(self):
        c = _Config()
        c.box[:] = [float(x) for x in self.box]
        c.nb[:] = [int(x) for x in self.nb]
        c.ratio = int(self.ratio)
        c.rho_f, c.mu_f, c.rho_p = float(self.rho_f), float(self.mu_f), float(self.rho_p)
        c.eps_min, c.phi_fp64 = float(self.eps_min), float(self.phi_fp64)
        c.deposit, c.precision, c.vel_source = int(self.deposit), int(self.precision), int(self.vel_source)
        c.advect, c.dt, c.max_particles = int(self.advect), float(self.dt), int(self.max_particles)
        c.mlp_tol, c.mlp_period = float(self.mlp_tol), int(self.mlp_period)
        c.semi_implicit = int(self.semi_implicit)
        c.vof, c.rho_f2, c.mu_f2 = int(self.vof), float(self.rho_f2), float(self.mu_f2)
        return c

    @property
    def n_bulk(self):
        return int(self.nb[0]) * int(self.nb[1]) * int(self.nb[2])

    @property
    def nf(self):
        return tuple(int(n) * int(self.ratio) for n in self.nb)

    @property
    def n_fine(self):
        return self.n_bulk * int(self.ratio) ** 3

    @property
    def dtype(self):
        return torch.float64 if self.precision == COUPLE_FP64 else torch.float32


def couple_last_error(h):
    s = _lib.couple_last_error(h)
    return s.decode() if s else ""


def _check(code, h):
    if code != COUPLE_OK:
        raise CoupleError(code, couple_last_error(h))


_HANDLE_CFG = {}   # handle address -> its Config (for the argument checks)


def couple_init(cfg: Config):
    """Validate ``cfg`` and allocate the library scratch; returns the handle."""
    h = C.c_void_p()
    c = cfg.to_c()
    code = _lib.couple_init(C.byref(c), C.byref(h))
    _check(code, None)
    _HANDLE_CFG[h.value] = Config(**cfg.__dict__)
    return h


def couple_free(h):
    if h is not None:
        _HANDLE_CFG.pop(h.value, None)
        _check(_lib.couple_free(h), None)


def _ptr(t):
    return None if t is None else t.data_ptr()


# ---- argument checks ------------------------------------------------------------
# The kernels index every array by sizes taken from the configuration, so a
# tensor of the wrong size, type, device or layout would be read or written out of
# bounds (or reinterpreted).  Every tensor is checked before the library sees its
# address; a failure raises ArgumentError (a ValueError) and nothing is launched.

def check_tensor(name, t, dtype, numel, device=None, optional=False, require_gpu=True, align=16, why=""):
    """Check one argument: a torch tensor on ``device`` (a GPU unless
    ``require_gpu`` is False) of ``dtype`` with ``numel`` elements, C-contiguous
    and ``align``-byte aligned.  ``None`` is accepted when ``optional``; ``why``
    says what makes a missing argument required."""
    if t is None:
        if optional:
            return
        raise ArgumentError(f"{name}: required{' ' + why if why else ''}, got None")
    if not isinstance(t, torch.Tensor):
        raise ArgumentError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if require_gpu and t.device.type != "cuda":
        raise ArgumentError(f"{name}: must be on a GPU, is on {t.device}")
    if device is not None and t.device != device:
        raise ArgumentError(f"{name}: on {t.device}, the other arguments are on {device}")
    if t.dtype != dtype:
        raise ArgumentError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.numel() != numel:
        raise ArgumentError(f"{name}: {t.numel()} elements (shape {tuple(t.shape)}), expected {numel}")
    if not t.is_contiguous():
        raise ArgumentError(f"{name}: not contiguous (a strided view); pass .contiguous()")
    if numel and align and t.data_ptr() % align:
        raise ArgumentError(f"{name}: data is not {align}-byte aligned (an offset view?)")


def validate_step(cfg, inputs, outputs, require_gpu=True):
    """Check the tensors of one couple_step call against the configuration
    (sizes, dtypes, devices, layout); raises ValueError."""
    n = inputs.get("n")
    if not isinstance(n, int) or n < 0:
        raise ArgumentError(f"n: expected an int >= 0, got {n!r}")
    if n > int(cfg.max_particles):
        raise ArgumentError(f"n = {n} exceeds max_particles = {cfg.max_particles}", COUPLE_ECAPACITY)
    ft, it = cfg.dtype, torch.int32
    nb, nf = cfg.n_bulk, cfg.n_fine
    dev = None
    for k in ("pos", "fine_u"):
        t = inputs.get(k)
        if isinstance(t, torch.Tensor):
            dev = t.device
            break
    kw = dict(device=dev, require_gpu=require_gpu)
    has_n = n > 0
    check_tensor("pos", inputs.get("pos"), ft, 3 * n, optional=not has_n, **kw)
    check_tensor("vel", inputs.get("vel"), ft, 3 * n, optional=not has_n, **kw)
    check_tensor("diam", inputs.get("diam"), ft, n, optional=not has_n, **kw)
    for k in ("fine_u", "fine_v", "fine_w", "fine_p"):
        check_tensor(k, inputs.get(k), ft, nf, **kw)
    check_tensor("uf_given", inputs.get("uf_given"), ft, 3 * n,
                 optional=not (has_n and cfg.vel_source == COUPLE_VEL_GIVEN), why="with vel_source GIVEN", **kw)
    check_tensor("fine_alpha", inputs.get("fine_alpha"), ft, nf, optional=not cfg.vof, why="with vof = 1", **kw)
    o = outputs
    check_tensor("drag", o.get("drag"), ft, 3 * n, optional=not has_n, **kw)
    check_tensor("beta", o.get("beta"), ft, n, optional=True, **kw)
    check_tensor("cell", o.get("cell"), it, n, optional=not has_n, **kw)
    check_tensor("perm", o.get("perm"), it, n, optional=not has_n, **kw)
    check_tensor("count", o.get("count"), it, nb, **kw)
    check_tensor("start", o.get("start"), it, nb + 1, **kw)
    for k, m in (("bulk_phi", 1), ("bulk_F", 3), ("bulk_U", 3), ("bulk_P", 1), ("bulk_G", 3)):
        check_tensor(k, o.get(k), ft, m * nb, **kw)
    check_tensor("fine_eps", o.get("fine_eps"), ft, nf, **kw)
    check_tensor("fine_F", o.get("fine_F"), ft, 3 * nf, **kw)
    check_tensor("diag", o.get("diag"), torch.float64, DIAG_LEN, **kw)
    check_tensor("uf", o.get("uf"), ft, 3 * n, optional=True, **kw)
    semi = bool(cfg.semi_implicit)
    ws = "with semi_implicit = 1"
    check_tensor("bulk_K", o.get("bulk_K"), ft, nb, optional=not semi, why=ws, **kw)
    check_tensor("bulk_KU", o.get("bulk_KU"), ft, 3 * nb, optional=not semi, why=ws, **kw)
    check_tensor("fine_K", o.get("fine_K"), ft, nf, optional=not semi, why=ws, **kw)
    check_tensor("fine_KU", o.get("fine_KU"), ft, 3 * nf, optional=not semi, why=ws, **kw)
    check_tensor("bulk_alpha", o.get("bulk_alpha"), ft, nb, optional=not cfg.vof, why="with vof = 1", **kw)


def couple_step(h, inputs: dict, outputs: dict, stream=None):
    """Enqueue one coupling step.  ``inputs``/``outputs`` map the field names of
    ``couple_inputs``/``couple_outputs`` to device tensors (or None).  Every
    tensor is checked against the handle's configuration first (ValueError)."""
    cfg = _HANDLE_CFG.get(getattr(h, "value", None))
    if cfg is None:
        raise ArgumentError("couple_step: not a live handle of couple_init")
    validate_step(cfg, inputs, outputs)
    i = _Inputs()
    i.n = int(inputs["n"])
    i.step = int(inputs.get("step", 0))
    for k in ("pos", "vel", "diam", "fine_u", "fine_v", "fine_w", "fine_p", "uf_given", "fine_alpha"):
        setattr(i, k, _ptr(inputs.get(k)))
    o = _Outputs()
    for k, _ in _Outputs._fields_:
        setattr(o, k, _ptr(outputs.get(k)))
    _check(_lib.couple_step(h, C.byref(i), C.byref(o), _stream(stream)), h)


NOALLOC_SCRATCH_BYTES = 64 << 20   # COUPLE_NOALLOC_SCRATCH_BYTES


def couple_step_noalloc(cfg: Config, inputs: dict, outputs: dict, stream=None):
    """The coupling step without a handle and without allocation (the library's
    static scratch; see couple_step_noalloc in include/couple.h).  Tensors are
    checked as for couple_step, with no particle capacity other than the
    scratch's."""
    chk = Config(**{**cfg.__dict__, "max_particles": max(int(inputs.get("n", 0)), int(cfg.max_particles))})
    validate_step(chk, inputs, outputs)
    c = cfg.to_c()
    i = _Inputs()
    i.n = int(inputs["n"])
    i.step = int(inputs.get("step", 0))
    for k in ("pos", "vel", "diam", "fine_u", "fine_v", "fine_w", "fine_p", "uf_given", "fine_alpha"):
        setattr(i, k, _ptr(inputs.get(k)))
    o = _Outputs()
    for k, _ in _Outputs._fields_:
        setattr(o, k, _ptr(outputs.get(k)))
    _check(_lib.couple_step_noalloc(C.byref(c), C.byref(i), C.byref(o), _stream(stream)), None)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    elif isinstance(stream, torch.cuda.Stream):
        stream = stream.cuda_stream
    return C.c_void_p(stream)


def hbmref(kind, src, dst, value=0.0, stream=None):
    """One pass of a streaming reference kernel (include/couple_hbmref.h) over
    float32 device tensors: COUPLE_HBMREF_READ scans ``src`` (4 k floats) and
    sets the one-element int32 ``dst`` to 1 if it holds a NaN or an infinity
    (the caller clears it); COUPLE_HBMREF_WRITE fills ``dst`` with ``value``;
    COUPLE_HBMREF_COPY copies ``src`` to ``dst``."""
    if kind not in (COUPLE_HBMREF_READ, COUPLE_HBMREF_WRITE, COUPLE_HBMREF_COPY):
        raise ArgumentError(f"kind: expected one of 0, 1, 2, got {kind!r}")
    ref = dst if kind == COUPLE_HBMREF_WRITE else src
    if not isinstance(ref, torch.Tensor) or ref.numel() % 4:
        raise ArgumentError("the buffer must be a float32 tensor of a multiple of 4 elements")
    n16 = ref.numel() // 4
    dev = ref.device
    if kind != COUPLE_HBMREF_WRITE:
        check_tensor("src", src, torch.float32, 4 * n16, device=dev)
    if kind == COUPLE_HBMREF_READ:
        check_tensor("dst", dst, torch.int32, 1, device=dev, align=4)
    else:
        check_tensor("dst", dst, torch.float32, 4 * n16, device=dev)
    _check(_lib.couple_hbmref(kind, _ptr(src), _ptr(dst), n16, float(value), _stream(stream)), None)


def couple_timing_begin(h, max_steps):
    """Start per-kernel event recording for at most ``max_steps`` steps."""
    _check(_lib.couple_timing_begin(h, int(max_steps)), h)


def couple_timing_end(h):
    """Stop recording; returns {kernel name: (launches, total milliseconds)}."""
    stats = (_KernelStat * 64)()
    n = C.c_int32(0)
    _check(_lib.couple_timing_end(h, stats, 64, C.byref(n)), h)
    return {stats[i].name.decode(): (int(stats[i].launches), float(stats[i].total_ms)) for i in range(n.value)}


def alloc_outputs(cfg: Config, n: int, device="cuda", beta=True, uf=False):
    """Device tensors for every output of a step with ``n`` particles (``uf``:
    also the fluid velocity used by the drag; the K/KU fields when the
    configuration asks for the semi-implicit split)."""
    dt = cfg.dtype
    nb, nf = cfg.nb, cfg.nf
    e = dict(device=device)
    semi = bool(cfg.semi_implicit)
    return {
        "drag": torch.empty((n, 3), dtype=dt, **e),
        "beta": torch.empty((n,), dtype=dt, **e) if beta else None,
        "cell": torch.empty((n,), dtype=torch.int32, **e),
        "perm": torch.empty((n,), dtype=torch.int32, **e),
        "count": torch.empty((nb[2], nb[1], nb[0]), dtype=torch.int32, **e),
        "start": torch.empty((cfg.n_bulk + 1,), dtype=torch.int32, **e),
        "bulk_phi": torch.empty((nb[2], nb[1], nb[0]), dtype=dt, **e),
        "bulk_F": torch.empty((3, nb[2], nb[1], nb[0]), dtype=dt, **e),
        "bulk_U": torch.empty((3, nb[2], nb[1], nb[0]), dtype=dt, **e),
        "bulk_P": torch.empty((nb[2], nb[1], nb[0]), dtype=dt, **e),
        "bulk_G": torch.empty((3, nb[2], nb[1], nb[0]), dtype=dt, **e),
        "fine_eps": torch.empty((nf[2], nf[1], nf[0]), dtype=dt, **e),
        "fine_F": torch.empty((3, nf[2], nf[1], nf[0]), dtype=dt, **e),
        "diag": torch.empty((DIAG_LEN,), dtype=torch.float64, **e),
        "uf": torch.empty((n, 3), dtype=dt, **e) if uf else None,
        "bulk_K": torch.empty((nb[2], nb[1], nb[0]), dtype=dt, **e) if semi else None,
        "bulk_KU": torch.empty((3, nb[2], nb[1], nb[0]), dtype=dt, **e) if semi else None,
        "fine_K": torch.empty((nf[2], nf[1], nf[0]), dtype=dt, **e) if semi else None,
        "fine_KU": torch.empty((3, nf[2], nf[1], nf[0]), dtype=dt, **e) if semi else None,
        "bulk_alpha": torch.empty((nb[2], nb[1], nb[0]), dtype=dt, **e) if cfg.vof else None,
    }


def diag_dict(diag_tensor):
    d = diag_tensor.detach().cpu().tolist()
    return {"V_tot": d[0], "V_dep": d[1], "sum_Fp": d[2:5], "S_b": d[5:8], "S_f": d[8:11], "E_f": d[11],
            "n_clamped": d[12], "n_outside": d[13], "max_phi": d[14], "n_fallback": d[15],
            "mlp_err2": d[16], "mlp_ref2": d[17], "mlp_nsamp": d[18], "K_p": d[19], "KU_p": d[20:23],
            "K_b": d[23], "KU_b": d[24:27], "K_f": d[27], "KU_f": d[28:31]}


class Coupler:
    """A handle plus its outputs.  ``step`` takes device tensors of the handle's
    dtype: pos [n,3], vel [n,3], diam [n], fine fields [nfz,nfy,nfx] (and the
    fine liquid fraction ``alpha`` when the configuration has ``vof``)."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.h = couple_init(cfg)
        self.out = None

    def step(self, pos, vel, diam, fine, uf_given=None, out=None, beta=True, stream=None, step=0, uf=False,
             alpha=None):
        n = pos.shape[0]
        if out is None:
            if (self.out is None or self.out["drag"].shape[0] != n or (uf and self.out["uf"] is None)):
                self.out = alloc_outputs(self.cfg, n, device=pos.device, beta=beta, uf=uf)
            out = self.out
        inputs = {"n": n, "pos": pos, "vel": vel, "diam": diam, "fine_u": fine[0], "fine_v": fine[1],
                  "fine_w": fine[2], "fine_p": fine[3], "uf_given": uf_given, "step": step, "fine_alpha": alpha}
        couple_step(self.h, inputs, out, stream=stream)
        return out

    def close(self):
        if self.h is not None:
            couple_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned velocity surrogate (include/couple_mlp.h) -------------------------

def couple_mlp_last_error(m):
    s = _lib.couple_mlp_last_error(m)
    return s.decode() if s else ""


def _mcheck(code, m):
    if code != COUPLE_OK:
        raise CoupleError(code, couple_mlp_last_error(m))


def _host(a, dtype):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def couple_mlp_init(max_batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    c = _MlpConfig(int(max_batch), float(lr), float(beta1), float(beta2), float(eps))
    m = C.c_void_p()
    _mcheck(_lib.couple_mlp_init(C.byref(c), C.byref(m)), None)
    return m


def couple_mlp_free(m):
    if m is not None:
        _mcheck(_lib.couple_mlp_free(m), None)


def couple_set_mlp(h, m):
    _check(_lib.couple_set_mlp(h, m), h)


def couple_mlp_features(cfg: Config, pos, diam, bulk_phi, bulk_U, bulk_G, feat, u_fine=None, sel=None,
                        u_bulk=None, resid=None, stream=None):
    """Raw surrogate features (and optionally bulk velocity and residual) of the
    particles ``sel`` (all when None) into device tensors."""
    c = cfg.to_c()
    if not isinstance(pos, torch.Tensor) or pos.dim() != 2:
        raise ArgumentError("pos: expected a [n, 3] tensor")
    n = pos.shape[0]
    nsel = n if sel is None else sel.numel()
    f32, nb = torch.float32, cfg.n_bulk
    kw = dict(device=pos.device, align=4)   # element-wise accesses: any 4-byte offset will do
    check_tensor("pos", pos, f32, 3 * n, **kw)
    check_tensor("diam", diam, f32, n, **kw)
    check_tensor("bulk_phi", bulk_phi, f32, nb, **kw)
    check_tensor("bulk_U", bulk_U, f32, 3 * nb, **kw)
    check_tensor("bulk_G", bulk_G, f32, 3 * nb, **kw)
    check_tensor("feat", feat, f32, MLP_NFEAT * nsel, **kw)
    check_tensor("u_fine", u_fine, f32, 3 * n, optional=resid is None, **kw)
    check_tensor("sel", sel, torch.int32, nsel, optional=True, **kw)
    check_tensor("u_bulk", u_bulk, f32, 3 * nsel, optional=True, **kw)
    check_tensor("resid", resid, f32, 3 * nsel, optional=True, **kw)
    _mcheck(_lib.couple_mlp_features(C.byref(c), n, _ptr(pos), _ptr(diam), _ptr(bulk_phi), _ptr(bulk_U),
                                     _ptr(bulk_G), _ptr(u_fine), _ptr(sel), nsel, _ptr(feat), _ptr(u_bulk),
                                     _ptr(resid), _stream(stream)), None)


class Mlp:
    """A surrogate network handle (device state owned by the library)."""

    def __init__(self, max_batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = couple_mlp_init(max_batch, lr, beta1, beta2, eps)
        self.max_batch = int(max_batch)

    def set_params(self, params):
        a, p = _host(params, "float32")
        if a.size != MLP_NPARAM:
            raise ArgumentError(f"params: {a.size} values, expected {MLP_NPARAM}")
        _mcheck(_lib.couple_mlp_set_params(self.m, p), self.m)

    def set_norm(self, mean, std, scale):
        a, pa = _host(mean, "float64")
        b, pb = _host(std, "float64")
        c, pc = _host(scale, "float64")
        _mcheck(_lib.couple_mlp_set_norm(self.m, pa, pb, pc), self.m)

    def _rows(self, feat, resid=None, limit=True):
        if not isinstance(feat, torch.Tensor) or feat.dim() != 2:
            raise ArgumentError("feat: expected a [rows, 193] tensor")
        n = feat.shape[0]
        if limit and n > self.max_batch:
            raise ArgumentError(f"feat: {n} rows exceed max_batch = {self.max_batch}")
        # rows are read element by element: any 4-byte offset (a slice of a pool) will do
        check_tensor("feat", feat, torch.float32, MLP_NFEAT * n, align=4)
        check_tensor("resid", resid, torch.float32, 3 * n, device=feat.device, optional=True, align=4)
        return n

    def fit_norm(self, feat, resid, stream=None):
        self._rows(feat, resid, limit=False)
        if resid is None:
            raise ArgumentError("resid: required")
        _mcheck(_lib.couple_mlp_fit_norm(self.m, _ptr(feat), _ptr(resid), feat.shape[0], _stream(stream)), self.m)

    def get_state(self):
        import numpy as np
        p = np.empty(MLP_NPARAM, np.float32)
        mm = np.empty(MLP_NPARAM, np.float32)
        vv = np.empty(MLP_NPARAM, np.float32)
        t = C.c_int64(0)
        mean = np.empty(MLP_NFEAT)
        std = np.empty(MLP_NFEAT)
        sc = np.empty(3)
        _mcheck(_lib.couple_mlp_get_state(self.m, p.ctypes.data, mm.ctypes.data, vv.ctypes.data, C.byref(t),
                                          mean.ctypes.data, std.ctypes.data, sc.ctypes.data), self.m)
        return {"params": p, "m": mm, "v": vv, "step": t.value, "mean": mean, "std": std, "scale": sc}

    def set_state(self, st):
        arrs = [_host(st[k], "float32") for k in ("params", "m", "v")] + \
               [_host(st[k], "float64") for k in ("mean", "std", "scale")]
        _mcheck(_lib.couple_mlp_set_state(self.m, arrs[0][1], arrs[1][1], arrs[2][1], int(st["step"]), arrs[3][1],
                                          arrs[4][1], arrs[5][1]), self.m)

    def forward(self, feat, y, stream=None):
        n = self._rows(feat)
        check_tensor("y", y, torch.float32, 3 * n, device=feat.device, align=4)
        _mcheck(_lib.couple_mlp_forward(self.m, _ptr(feat), feat.shape[0], _ptr(y), _stream(stream)), self.m)

    def _batch(self, feat, resid, B, idx):
        n = self._rows(feat, resid, limit=False)
        if resid is None:
            raise ArgumentError("resid: required")
        if idx is None and int(B) > n:
            raise ArgumentError(f"B = {B} exceeds the {n} rows")
        check_tensor("idx", idx, torch.int32, int(B), device=feat.device, optional=True, align=4)

    def grads(self, feat, resid, B, grads, idx=None, loss=None, stream=None):
        self._batch(feat, resid, B, idx)
        check_tensor("grads", grads, torch.float32, MLP_NPARAM, device=feat.device)
        check_tensor("loss", loss, torch.float32, 1, device=feat.device, optional=True)
        _mcheck(_lib.couple_mlp_grads(self.m, _ptr(feat), _ptr(resid), feat.shape[0], _ptr(idx), int(B),
                                      _ptr(grads), _ptr(loss), _stream(stream)), self.m)

    def adam(self, grads, stream=None):
        check_tensor("grads", grads, torch.float32, MLP_NPARAM)
        _mcheck(_lib.couple_mlp_adam(self.m, _ptr(grads), _stream(stream)), self.m)

    def train_step(self, feat, resid, B, idx=None, loss=None, stream=None):
        self._batch(feat, resid, B, idx)
        check_tensor("loss", loss, torch.float32, 1, device=feat.device, optional=True)
        _mcheck(_lib.couple_mlp_train_step(self.m, _ptr(feat), _ptr(resid), feat.shape[0], _ptr(idx), int(B),
                                           _ptr(loss), _stream(stream)), self.m)

    def close(self):
        if self.m is not None:
            couple_mlp_free(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- grid-to-grid transfer between non-nested grids (include/couple_remap.h) ----

def _rcheck(code, r):
    if code != COUPLE_OK:
        s = _lib.couple_remap_last_error(r)
        raise CoupleError(code, s.decode() if s else "")


class Remap:
    """Volume-weighted transfer from a sender grid to a receiver grid over the
    same box.  ``src_nodes`` / ``dst_nodes``: three 1-D arrays of node
    coordinates (x, y, z) of rectilinear cell-centred grids."""

    def __init__(self, src_nodes, dst_nodes, precision=COUPLE_FP32_WIDE):
        import numpy as np
        self.ns = [len(a) - 1 for a in src_nodes]
        self.nd = [len(a) - 1 for a in dst_nodes]
        self.precision = int(precision)
        ns, pns = _host(self.ns, "int32")
        nd, pnd = _host(self.nd, "int32")
        sn, psn = _host(np.concatenate([np.asarray(a, np.float64) for a in src_nodes]), "float64")
        dn, pdn = _host(np.concatenate([np.asarray(a, np.float64) for a in dst_nodes]), "float64")
        r = C.c_void_p()
        _rcheck(_lib.couple_remap_init(pns, psn, pnd, pdn, self.precision, C.byref(r)), None)
        self.r = r

    @property
    def dtype(self):
        return torch.float64 if self.precision == COUPLE_FP64 else torch.float32

    def apply(self, src, dst=None, stream=None):
        """src: device tensor [..., nz, ny, nx] of the sender grid (leading dims =
        fields); returns dst [..., nz', ny', nx'] of the receiver grid."""
        nsrc = self.ns[0] * self.ns[1] * self.ns[2]
        ndst = self.nd[0] * self.nd[1] * self.nd[2]
        if not isinstance(src, torch.Tensor) or src.numel() == 0 or src.numel() % nsrc:
            raise ArgumentError(f"src: expected a whole number (>= 1) of sender fields of {nsrc} cells")
        nf = src.numel() // nsrc
        check_tensor("src", src, self.dtype, nf * nsrc)
        lead = tuple(src.shape[:-3]) if src.dim() > 3 else ()
        if dst is None:
            dst = torch.empty(lead + (self.nd[2], self.nd[1], self.nd[0]), dtype=self.dtype, device=src.device)
        check_tensor("dst", dst, self.dtype, nf * ndst, device=src.device)
        _rcheck(_lib.couple_remap_apply(self.r, _ptr(src), _ptr(dst), nf, _stream(stream)), self.r)
        return dst

    def info(self):
        ax = (C.c_int64 * 3)()
        tot = C.c_int64(0)
        _rcheck(_lib.couple_remap_info(self.r, ax, C.byref(tot)), self.r)
        return list(ax), int(tot.value)

    def close(self):
        if getattr(self, "r", None) is not None:
            _lib.couple_remap_free(self.r)
            self.r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- transfer between grids of arbitrary axis-aligned cells (include/couple_boxmap.h) ----

class BoxMap:
    """Volume-weighted transfer from a sender grid to a receiver grid, each an
    [n, 6] array of axis-aligned cells (x0, x1, y0, y1, z0, z1), through a CSR
    overlap map built once (host, FP64) and applied on the device."""

    def __init__(self, sender_boxes, receiver_boxes, precision=COUPLE_FP32_WIDE):
        import numpy as np
        sb, psb = _host(np.asarray(sender_boxes, np.float64).reshape(-1, 6), "float64")
        rb, prb = _host(np.asarray(receiver_boxes, np.float64).reshape(-1, 6), "float64")
        self.ns, self.nr = sb.shape[0], rb.shape[0]
        self.precision = int(precision)
        m = C.c_void_p()
        code = _lib.couple_boxmap_init(self.ns, psb, self.nr, prb, self.precision, C.byref(m))
        if code != COUPLE_OK:
            s = _lib.couple_boxmap_last_error(None)
            raise CoupleError(code, s.decode() if s else "")
        self.m = m

    @property
    def dtype(self):
        return torch.float64 if self.precision == COUPLE_FP64 else torch.float32

    def apply(self, src, dst=None, stream=None):
        """src: device tensor [nfields, ns] (or [ns]); returns dst [nfields, nr]
        (or [nr])."""
        if not isinstance(src, torch.Tensor) or src.numel() == 0 or src.numel() % self.ns:
            raise ArgumentError(f"src: expected a whole number (>= 1) of sender fields of {self.ns} cells")
        nf = src.numel() // self.ns
        check_tensor("src", src, self.dtype, nf * self.ns)
        if dst is None:
            dst = torch.empty((nf, self.nr) if src.dim() > 1 else (self.nr,), dtype=self.dtype, device=src.device)
        check_tensor("dst", dst, self.dtype, nf * self.nr, device=src.device)
        code = _lib.couple_boxmap_apply(self.m, _ptr(src), _ptr(dst), nf, _stream(stream))
        if code != COUPLE_OK:
            s = _lib.couple_boxmap_last_error(self.m)
            raise CoupleError(code, s.decode() if s else "")
        return dst

    def info(self):
        nnz, mr = C.c_int64(0), C.c_int64(0)
        _lib.couple_boxmap_info(self.m, C.byref(nnz), C.byref(mr))
        return int(nnz.value), int(mr.value)

    def close(self):
        if getattr(self, "m", None) is not None:
            _lib.couple_boxmap_free(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- partitioned step (couple_part_* of include/couple.h) ----------------------

class Part:
    """The coupling step on ``nparts`` co-located z-slabs of one device, with the
    halos exchanged through the static neighbour-to-neighbour communication
    matrix, directly (``exchange=COUPLE_EXCHANGE_DISTRIBUTED``) or through a root
    buffer (``COUPLE_EXCHANGE_GATHER_SCATTER``).  ``step`` takes and returns what
    ``Coupler.step`` does."""

    def __init__(self, cfg: Config, nparts: int):
        self.cfg = cfg
        self.nparts = int(nparts)
        c = cfg.to_c()
        p = C.c_void_p()
        code = _lib.couple_part_init(C.byref(c), self.nparts, C.byref(p))
        if code != COUPLE_OK:
            s = _lib.couple_part_last_error(None)
            raise CoupleError(code, s.decode() if s else "")
        self.p = p
        self.out = None

    def step(self, pos, vel, diam, fine, out=None, exchange=COUPLE_EXCHANGE_DISTRIBUTED, stream=None, step=0,
             beta=True, uf=False):
        n = pos.shape[0]
        if out is None:
            if self.out is None or self.out["drag"].shape[0] != n or (uf and self.out["uf"] is None):
                self.out = alloc_outputs(self.cfg, n, device=pos.device, beta=beta, uf=uf)
            out = self.out
        inputs = {"n": n, "pos": pos, "vel": vel, "diam": diam, "fine_u": fine[0], "fine_v": fine[1],
                  "fine_w": fine[2], "fine_p": fine[3], "step": step}
        validate_step(self.cfg, inputs, out)
        i = _Inputs()
        i.n = int(n)
        i.step = int(step)
        for k in ("pos", "vel", "diam", "fine_u", "fine_v", "fine_w", "fine_p"):
            setattr(i, k, _ptr(inputs.get(k)))
        o = _Outputs()
        for k, _ in _Outputs._fields_:
            setattr(o, k, _ptr(out.get(k)))
        code = _lib.couple_part_step(self.p, C.byref(i), C.byref(o), int(exchange), _stream(stream))
        if code != COUPLE_OK:
            s = _lib.couple_part_last_error(self.p)
            raise CoupleError(code, s.decode() if s else "")
        return out

    def comm_matrix(self):
        """[nparts, nparts] int64 array: entry (i, j) is the bytes slab j sends to
        slab i in one step."""
        import numpy as np
        m = np.zeros((self.nparts, self.nparts), np.int64)
        code = _lib.couple_part_comm_matrix(self.p, m.ctypes.data_as(C.c_void_p))
        if code != COUPLE_OK:
            raise CoupleError(code, "couple_part_comm_matrix failed")
        return m

    def close(self):
        if getattr(self, "p", None) is not None:
            _lib.couple_part_free(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
