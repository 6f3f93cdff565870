"""Thin ctypes binding of libyyg.so (include/yyg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device arrays are passed as torch CUDA tensors (their data pointer
and the current stream); host arrays as numpy arrays.  Raises when the
library has not been built — there is no fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libyyg.so")

FP64, FP32, BF16X3, FP16X2 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x2": FP16X2}

TABLE_WEIGHTS, TABLE_THETA, TABLE_PHI, TABLE_RADIAL, TABLE_CROSS, TABLE_ROTATION = 0, 1, 2, 3, 4, 5
METHODS = {"dense": 0, "separable": 1}
# yyg_status
OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_READY, ERR_UNSUPPORTED, ERR_NONFINITE = 0, -1, -2, -3, -4, -5, -6
GRID_YINYANG, GRID_POLAR = 0, 1
KINDS = {"yinyang": GRID_YINYANG, "polar": GRID_POLAR}

EXPORTS = [
    "yyg_grid_create", "yyg_grid_create_res", "yyg_grid_dims", "yyg_prepare",
    "yyg_upload_rho", "yyg_solve", "yyg_get_moments", "yyg_get_weights",
    "yyg_grid_destroy", "yyg_host_table", "yyg_set_timing", "yyg_get_timing",
    "yyg_batch_create", "yyg_batch_solve", "yyg_batch_destroy", "yyg_status_string",
    "yyg_autotune", "yyg_plan_info", "yyg_plan_config", "yyg_batch_autotune", "yyg_batch_info",
    "yyg_batch_profile", "yyg_set_method", "yyg_grid_kind", "yyg_sep_config", "yyg_sep_info",
    "yyg_sep_kernel", "yyg_sep_phase", "yyg_solve_noalloc", "yyg_sep_lp_kernel", "yyg_sep_lp_config",
    "yyg_set_check_finite", "yyg_device_bytes", "yyg_sep_variant_count",
]


class YygError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {lib().yyg_status_string(status).decode()} ({status})")


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("n_r", ctypes.c_int),
        ("r_edges", ctypes.POINTER(ctypes.c_double)),
        ("n_theta", ctypes.c_int),
        ("n_phi", ctypes.c_int),
        ("delta_theta", ctypes.c_double),
        ("delta_phi", ctypes.c_double),
        ("lmax", ctypes.c_int),
        ("G", ctypes.c_double),
        ("kind", ctypes.c_int),
    ]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1806_04593_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname; loading it
        # first makes libyyg bind to that copy, so the process has a single
        # HIP runtime (two copies cannot share the device, streams or memory).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double)
        L.yyg_grid_create.argtypes = [ctypes.POINTER(GridDesc), i, ctypes.POINTER(vp)]
        L.yyg_grid_create_res.argtypes = [i, dp, d, i, d, i, ctypes.POINTER(vp)]
        L.yyg_grid_dims.argtypes = [vp] + [ctypes.POINTER(i)] * 4
        L.yyg_grid_kind.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.yyg_prepare.argtypes = [vp, i]
        L.yyg_upload_rho.argtypes = [vp, vp, i, vp]
        L.yyg_solve.argtypes = [vp, vp, i, i, vp]
        L.yyg_get_moments.argtypes = [vp, dp]
        L.yyg_get_weights.argtypes = [vp, dp]
        L.yyg_grid_destroy.argtypes = [vp]
        L.yyg_host_table.argtypes = [ctypes.POINTER(GridDesc), i, dp, ctypes.c_size_t]
        L.yyg_set_timing.argtypes = [vp, i]
        L.yyg_get_timing.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_long), i]
        L.yyg_batch_create.argtypes = [ctypes.POINTER(vp), i, i, ctypes.POINTER(vp)]
        L.yyg_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.yyg_batch_destroy.argtypes = [vp]
        L.yyg_batch_autotune.argtypes = [vp, vp]
        L.yyg_batch_info.argtypes = [vp, ctypes.POINTER(i), i]
        L.yyg_batch_profile.argtypes = [vp, vp, dp, i]
        L.yyg_set_method.argtypes = [vp, i]
        L.yyg_sep_config.argtypes = [vp, i, i]
        L.yyg_sep_info.argtypes = [vp, ctypes.POINTER(i), i]
        L.yyg_sep_kernel.argtypes = [vp, i, ctypes.c_char_p, ctypes.c_size_t]
        L.yyg_sep_phase.argtypes = [vp, i, vp, vp]
        L.yyg_solve_noalloc.argtypes = [vp, vp, vp, vp]
        L.yyg_sep_lp_kernel.argtypes = [vp, i, i, ctypes.c_char_p, ctypes.c_size_t]
        L.yyg_sep_lp_config.argtypes = [vp, i, i, i]
        L.yyg_set_check_finite.argtypes = [vp, i]
        L.yyg_device_bytes.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        L.yyg_sep_variant_count.argtypes = [i]
        L.yyg_autotune.argtypes = [vp, i, vp]
        L.yyg_plan_info.argtypes = [vp, i, ctypes.POINTER(i), i]
        L.yyg_plan_config.argtypes = [vp, i, i, i, i]
        L.yyg_status_string.argtypes = [i]
        L.yyg_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "yyg_status_string":
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def device_bytes():
    """Device memory the library holds in this process (yyg_device_bytes)."""
    n = ctypes.c_size_t(0)
    _check(lib().yyg_device_bytes(ctypes.byref(n)), "yyg_device_bytes")
    return int(n.value)


def _check(status, where):
    if status != 0:
        raise YygError(status, where)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_desc(r_edges, n_theta, n_phi, delta_theta, delta_phi, lmax, G, kind=GRID_YINYANG):
    r = np.ascontiguousarray(r_edges, dtype=np.float64)
    d = GridDesc(len(r) - 1, _dptr(r), int(n_theta), int(n_phi), float(delta_theta),
                 float(delta_phi), int(lmax), float(G), int(KINDS.get(kind, kind)))
    d._keep = r  # keep the radii alive with the descriptor
    return d


def _desc_of(desc):
    return make_desc(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"],
                     desc["delta_phi"], desc["lmax"], desc.get("G", 1.0), desc.get("kind", "yinyang"))


def host_table(desc, which):
    """Host-only table builder (no GPU needed); returns a numpy array."""
    d = _desc_of(desc)
    Q = (desc["lmax"] + 1) ** 2
    nang = desc["n_theta"] * desc["n_phi"]
    n_r = len(desc["r_edges"]) - 1
    shape = {TABLE_WEIGHTS: (desc["n_theta"], desc["n_phi"]),
             TABLE_THETA: (desc["n_theta"], Q),
             TABLE_PHI: (desc["n_phi"], Q),
             TABLE_RADIAL: (n_r, desc["lmax"] + 1, 4),
             TABLE_CROSS: (nang, 3),
             TABLE_ROTATION: (sum((2 * l + 1) ** 2 for l in range(desc["lmax"] + 1)),)}[which]
    shape = tuple(max(0, v) for v in shape)
    out = np.zeros(shape)
    buf = out if out.size else np.zeros(1)   # the library validates the sizes itself
    _check(lib().yyg_host_table(ctypes.byref(d), which, _dptr(buf), out.size), "yyg_host_table")
    return out


def device_array(t, shape, what, device=None):
    """Check that `t` is a C-contiguous torch CUDA float64 tensor of `shape`
    and return its device address.  The library cannot size-check a raw
    device pointer, so a wrong dtype, size or a host tensor is refused here,
    before any library call (ValueError, not an assert: -O keeps it)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch CUDA tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise ValueError(f"{what}: dtype {t.dtype}, expected torch.float64")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor on {t.device}, expected a CUDA (HIP) device tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what}: tensor on {t.device}, the plan is on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor is not contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def host_array(a, shape, what):
    """Check that `a` is a C-contiguous numpy float64 array of `shape`."""
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
        raise ValueError(f"{what}: expected a C-contiguous numpy float64 array")
    if a.shape != tuple(shape):
        raise ValueError(f"{what}: shape {a.shape}, expected {tuple(shape)}")
    return a.ctypes.data


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Grid:
    """A plan on one device: yyg_grid_create + the calls taking it."""

    def __init__(self, desc, device=0):
        d = _desc_of(desc)
        h = ctypes.c_void_p()
        _check(lib().yyg_grid_create(ctypes.byref(d), int(device), ctypes.byref(h)), "yyg_grid_create")
        self._h = h
        self.device = device
        n_r, n_t, n_p, Q = (ctypes.c_int() for _ in range(4))
        _check(lib().yyg_grid_dims(h, ctypes.byref(n_r), ctypes.byref(n_t), ctypes.byref(n_p), ctypes.byref(Q)),
               "yyg_grid_dims")
        self.n_r, self.n_theta, self.n_phi, self.Q = n_r.value, n_t.value, n_p.value, Q.value
        kind, patches = ctypes.c_int(), ctypes.c_int()
        _check(lib().yyg_grid_kind(h, ctypes.byref(kind), ctypes.byref(patches)), "yyg_grid_kind")
        self.kind, self.patches = kind.value, patches.value
        self.shape = (self.patches, self.n_r, self.n_theta, self.n_phi)

    @property
    def handle(self):
        return self._h

    def set_method(self, method):
        _check(lib().yyg_set_method(self._h, METHODS.get(method, method)), "yyg_set_method")

    def prepare(self, precision):
        _check(lib().yyg_prepare(self._h, PRECISIONS.get(precision, precision)), "yyg_prepare")

    def upload_rho(self, rho, stream=None):
        """rho: torch CUDA tensor (borrowed) or numpy array (copied)."""
        if isinstance(rho, np.ndarray):
            r = np.ascontiguousarray(rho, dtype=np.float64)
            ptr = host_array(r, self.shape, "upload_rho")
            self._host_rho = r
            _check(lib().yyg_upload_rho(self._h, ctypes.c_void_p(ptr), 0, _stream_handle(stream)),
                   "yyg_upload_rho")
        else:
            ptr = device_array(rho, self.shape, "upload_rho", self.device)
            self._dev_rho = rho
            _check(lib().yyg_upload_rho(self._h, ctypes.c_void_p(ptr), 1, _stream_handle(stream)),
                   "yyg_upload_rho")

    def solve(self, phi, precision="fp64", stream=None):
        """phi: preallocated torch CUDA float64 tensor (async) or numpy (sync)."""
        p = PRECISIONS.get(precision, precision)
        if isinstance(phi, np.ndarray):
            ptr = host_array(phi, self.shape, "solve")
            _check(lib().yyg_solve(self._h, ctypes.c_void_p(ptr), 0, p, _stream_handle(stream)), "yyg_solve")
        else:
            ptr = device_array(phi, self.shape, "solve", self.device)
            _check(lib().yyg_solve(self._h, ctypes.c_void_p(ptr), 1, p, _stream_handle(stream)), "yyg_solve")
        return phi

    def solve_noalloc(self, rho, phi, stream=None):
        """yyg_solve_noalloc: separable FP64 solve of device `rho` into
        device `phi` with the intermediates in the library's fixed scratch
        array (no allocation)."""
        rp = device_array(rho, self.shape, "solve_noalloc rho", self.device)
        pp = device_array(phi, self.shape, "solve_noalloc phi", self.device)
        _check(lib().yyg_solve_noalloc(self._h, ctypes.c_void_p(rp), ctypes.c_void_p(pp), _stream_handle(stream)),
               "yyg_solve_noalloc")
        return phi

    def set_check_finite(self, on=True):
        """yyg_set_check_finite: scan the density for NaN / infinity before
        every solve (YygError with status YYG_ERR_NONFINITE if found)."""
        _check(lib().yyg_set_check_finite(self._h, 1 if on else 0), "yyg_set_check_finite")

    def autotune(self, precision="fp64", stream=None):
        _check(lib().yyg_autotune(self._h, PRECISIONS.get(precision, precision), _stream_handle(stream)),
               "yyg_autotune")

    def plan_info(self, precision="fp64"):
        info = (ctypes.c_int * 7)()
        _check(lib().yyg_plan_info(self._h, PRECISIONS.get(precision, precision), info, 7), "yyg_plan_info")
        keys = ("var_ana", "split_ana", "var_syn", "bm_ana", "bn_ana", "bm_syn", "bn_syn")
        return dict(zip(keys, list(info)))

    def sep_config(self, phase, variant):
        _check(lib().yyg_sep_config(self._h, int(phase), int(variant)), "yyg_sep_config")

    def sep_variant_count(self, phase):
        """yyg_sep_variant_count: the length of phase `phase`'s variant range."""
        n = lib().yyg_sep_variant_count(int(phase))
        _check(min(n, 0), "yyg_sep_variant_count")
        return n

    def sep_info(self):
        v = (ctypes.c_int * 5)()
        _check(lib().yyg_sep_info(self._h, v, 5), "yyg_sep_info")
        return list(v)

    def sep_kernel(self, phase):
        buf = ctypes.create_string_buffer(256)
        _check(lib().yyg_sep_kernel(self._h, int(phase), buf, 256), "yyg_sep_kernel")
        return buf.value.decode()

    def sep_lp_kernel(self, precision, phase):
        buf = ctypes.create_string_buffer(256)
        _check(lib().yyg_sep_lp_kernel(self._h, PRECISIONS.get(precision, precision), int(phase), buf, 256),
               "yyg_sep_lp_kernel")
        return buf.value.decode()

    def sep_phase(self, phase, phi, stream=None):
        """Launch one separable phase alone (after a solve); phi: the torch
        CUDA float64 tensor phase 4 writes."""
        ptr = device_array(phi, self.shape, "sep_phase", self.device)
        _check(lib().yyg_sep_phase(self._h, int(phase), ctypes.c_void_p(ptr), _stream_handle(stream)),
               "yyg_sep_phase")

    def set_config(self, var_ana, split_ana, var_syn, precision="fp64"):
        _check(lib().yyg_plan_config(self._h, PRECISIONS.get(precision, precision), int(var_ana), int(split_ana),
                                     int(var_syn)), "yyg_plan_config")

    def moments(self):
        out = np.zeros((self.patches, self.n_r, self.Q))
        _check(lib().yyg_get_moments(self._h, _dptr(out)), "yyg_get_moments")
        return out

    def weights(self):
        out = np.zeros((self.n_theta, self.n_phi))
        _check(lib().yyg_get_weights(self._h, _dptr(out)), "yyg_get_weights")
        return out

    def set_timing(self, enable):
        _check(lib().yyg_set_timing(self._h, int(bool(enable))), "yyg_set_timing")

    def timing(self, n_slots=8):
        ms = np.zeros(n_slots)
        cnt = (ctypes.c_long * n_slots)()
        _check(lib().yyg_get_timing(self._h, _dptr(ms), cnt, n_slots), "yyg_get_timing")
        return ms, np.array(list(cnt))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yyg_grid_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched solves of several plans (yyg_batch_*)."""

    def __init__(self, grids, precision="fp64"):
        self.grids = list(grids)
        arr = (ctypes.c_void_p * len(self.grids))(*[g.handle.value for g in self.grids])
        h = ctypes.c_void_p()
        _check(lib().yyg_batch_create(arr, len(self.grids), PRECISIONS.get(precision, precision), ctypes.byref(h)),
               "yyg_batch_create")
        self._h = h
        self.precision = precision

    def solve(self, rhos, phis, stream=None):
        """rhos, phis: lists of torch CUDA float64 tensors, one per field."""
        n = len(self.grids)
        if len(rhos) != n or len(phis) != n:
            raise ValueError(f"batch solve: {len(rhos)} densities and {len(phis)} potentials for {n} fields")
        rp = [device_array(r, g.shape, f"batch rho[{f}]", g.device) for f, (g, r) in enumerate(zip(self.grids, rhos))]
        pp = [device_array(p, g.shape, f"batch phi[{f}]", g.device) for f, (g, p) in enumerate(zip(self.grids, phis))]
        self._keep = (list(rhos), list(phis))
        ra = (ctypes.c_void_p * n)(*rp)
        pa = (ctypes.c_void_p * n)(*pp)
        _check(lib().yyg_batch_solve(self._h, ra, pa, _stream_handle(stream)), "yyg_batch_solve")

    def autotune(self, stream=None):
        _check(lib().yyg_batch_autotune(self._h, _stream_handle(stream)), "yyg_batch_autotune")

    def profile(self, stream=None):
        """Per-phase milliseconds of one eager run: analysis, scan, synthesis, splits."""
        ms = np.zeros(4)
        _check(lib().yyg_batch_profile(self._h, _stream_handle(stream), _dptr(ms), 4), "yyg_batch_profile")
        return ms

    def info(self):
        info = (ctypes.c_int * 9)()
        _check(lib().yyg_batch_info(self._h, info, 9), "yyg_batch_info")
        return dict(zip(("fields", "precision", "var_ana", "var_syn", "items_ana", "items_syn", "var_theta_ana",
                         "var_rotation", "var_theta_syn"), list(info)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().yyg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
