"""ctypes binding of libtfocus (include/tfocus.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions carry the C names; descriptors may be given as dicts (the keys of
the C structs, enums as strings) and arrays as torch tensors (device memory,
passed by data_ptr on the current stream) or numpy arrays (host memory).
Failures raise ``TfError`` with the library's status and message.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libtfocus.so")
# kernel plans tuned on MI355X (tf_tune); used unless TFOCUS_PLAN_FILE is set
DEFAULT_PLANS = os.path.join(HERE, "plans", "gfx950.txt")

TF_OK, TF_EINVAL, TF_EUNSUPPORTED, TF_ENOMEM, TF_EDEVICE, TF_ESTATE, TF_EDOMAIN, TF_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "TF_OK", -1: "TF_EINVAL", -2: "TF_EUNSUPPORTED", -3: "TF_ENOMEM",
                -4: "TF_EDEVICE", -5: "TF_ESTATE", -6: "TF_EDOMAIN", -7: "TF_ENONFINITE"}
TF_F32, TF_F64 = 0, 1
ENVELOPES = {"cos2": 0, "gauss": 1, "spectral": 2}
TRANSVERSE = {"flattop": 0, "gauss": 1}
POLARIZATION = {"linear": 0, "radial": 1}
PRECISION = {"f32": TF_F32, "f64": TF_F64}


class TfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class tf_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("replicate_yz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("x_min", ctypes.c_double), ("y_min", ctypes.c_double), ("z_min", ctypes.c_double)]


class tf_pulse(ctypes.Structure):
    _fields_ = [("envelope", ctypes.c_int32), ("transverse", ctypes.c_int32),
                ("polarization", ctypes.c_int32), ("nfreq", ctypes.c_int32)] + \
               [(n, ctypes.c_double) for n in ("wavelength", "R0", "L", "ncycles", "f_number",
                                                 "theta", "eps", "P0", "pol_angle", "ellipticity",
                                                 "cep", "gdd", "tod", "bandwidth")] + \
               [("nbumps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("bumps", ctypes.POINTER(ctypes.c_double))]


class tf_pulse_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("theta", "A", "R_min", "R_max", "L", "D_min",
                                                "alpha_max", "D")] + \
               [("overlap", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class tf_window(ctypes.Structure):
    _fields_ = [("wx", ctypes.c_int32), ("wy", ctypes.c_int32), ("wz", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double)]


TRAIN_PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p)


class tf_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("lr_min_frac", ctypes.c_double), ("seed", ctypes.c_uint64), ("scale_targets", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("epoch_loss", ctypes.POINTER(ctypes.c_double)),
                ("progress", TRAIN_PROGRESS), ("progress_user", ctypes.c_void_p)]


_P = ctypes.c_void_p
_SIGS = {
    "tf_version": ([], ctypes.c_char_p),
    "tf_last_error": ([], ctypes.c_char_p),
    "tf_supported_length": ([ctypes.c_int32], ctypes.c_int32),
    "tf_pulse_geometry": ([ctypes.POINTER(tf_pulse), ctypes.POINTER(tf_pulse_info)], ctypes.c_int),
    "tf_layer_grid": ([ctypes.POINTER(tf_pulse), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(tf_grid)],
                      ctypes.c_int),
    "tf_create": ([ctypes.POINTER(tf_grid), ctypes.c_int32, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "tf_destroy": ([_P], ctypes.c_int),
    "tf_set_fields": ([_P, _P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "tf_get_fields": ([_P, _P, ctypes.c_int32], ctypes.c_int),
    "tf_state_ptr": ([_P, ctypes.POINTER(_P)], ctypes.c_int),
    "tf_set_pulse": ([_P, ctypes.POINTER(tf_pulse), ctypes.POINTER(tf_pulse_info)], ctypes.c_int),
    "tf_set_cutout": ([_P, ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "tf_advance": ([_P, ctypes.c_int64, ctypes.c_double], ctypes.c_int),
    "tf_advance_current": ([_P, _P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "tf_read_focal": ([_P, ctypes.POINTER(tf_window), _P, ctypes.c_int32], ctypes.c_int),
    "tf_diagnostics": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tf_advance_diagnosed": ([_P, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tf_time": ([_P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tf_get_grid": ([_P, ctypes.POINTER(tf_grid)], ctypes.c_int),
    "tf_batch_create": ([ctypes.POINTER(tf_grid), ctypes.POINTER(tf_pulse), ctypes.c_int32, ctypes.c_int32, _P,
                         ctypes.POINTER(_P)], ctypes.c_int),
    "tf_batch_run": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(tf_window),
                      _P, ctypes.c_int32], ctypes.c_int),
    "tf_batch_get_fields": ([_P, ctypes.c_int32, _P, ctypes.c_int32], ctypes.c_int),
    "tf_batch_destroy": ([_P], ctypes.c_int),
    "tf_set_plan_file": ([ctypes.c_char_p], ctypes.c_int),
    "tf_tune": ([ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                 ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tf_advance_noalloc": ([ctypes.POINTER(tf_grid), ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_double,
                            ctypes.c_int32, _P], ctypes.c_int),
    "tf_kernel_plan": ([ctypes.POINTER(tf_grid), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "tf_profile": ([_P, ctypes.c_int32], ctypes.c_int),
    "tf_profile_read": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "tf_fno_param_count": ([ctypes.c_int32], ctypes.c_int64),
    "tf_fno_phasor_weights": ([ctypes.POINTER(tf_pulse), ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
                              ctypes.c_int),
    "tf_fno_create": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "tf_fno_destroy": ([_P], ctypes.c_int),
    "tf_fno_set_params": ([_P, _P, ctypes.c_int32], ctypes.c_int),
    "tf_fno_get_params": ([_P, _P, ctypes.c_int32], ctypes.c_int),
    "tf_fno_forward": ([_P, _P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "tf_fno_infer": ([_P, _P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "tf_fno_loss_grad": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "tf_fno_train_step": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
                          ctypes.c_int),
    "tf_fno_train": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.POINTER(tf_train_cfg), ctypes.POINTER(ctypes.c_double)],
                     ctypes.c_int),
    "tf_fno_eval": ([_P, _P, _P, _P, ctypes.c_int64, _P], ctypes.c_int),
    "tf_fno_spectral_forward": ([_P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "tf_fno_spectral_inverse": ([_P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "tf_fno_save": ([_P, ctypes.c_char_p], ctypes.c_int),
    "tf_fno_set_period": ([_P, ctypes.c_int32], ctypes.c_int),
    "tf_fno_get_period": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "tf_fno_load": ([_P, ctypes.c_char_p], ctypes.c_int),
}

PASS_NAMES = ("x_forward", "y_forward", "z_step", "y_inverse", "x_inverse", "init", "readout", "other")

_lib = None


def load():
    """Load libtfocus.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with "
                               "`python -m paper_2010_00409_amd.build`")
        lib = ctypes.CDLL(LIBPATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        if not os.environ.get("TFOCUS_PLAN_FILE") and os.path.exists(DEFAULT_PLANS):
            lib.tf_set_plan_file(DEFAULT_PLANS.encode())
    return _lib


def exported_names():
    return list(_SIGS)


def _check(status):
    if status != TF_OK:
        raise TfError(status, load().tf_last_error().decode())


# ---- descriptor conversion ----------------------------------------------------

def grid_struct(g):
    if isinstance(g, tf_grid):
        return g
    return tf_grid(int(g["nx"]), int(g["ny"]), int(g["nz"]), int(g.get("replicate_yz", 0)), float(g["dx"]),
                   float(g["dy"]),
                   float(g["dz"]), float(g["x_min"]), float(g["y_min"]), float(g["z_min"]))


def grid_dict(s):
    d = {k: getattr(s, k) for k in ("nx", "ny", "nz", "dx", "dy", "dz", "x_min", "y_min", "z_min")}
    if s.replicate_yz:
        d["replicate_yz"] = 1
    return d


def pulse_struct(p):
    if isinstance(p, tf_pulse):
        return p
    s = tf_pulse()
    s.envelope = ENVELOPES[p["envelope"]]
    s.transverse = TRANSVERSE[p["transverse"]]
    s.polarization = POLARIZATION[p["polarization"]]
    s.nfreq = int(p.get("nfreq", 256))
    for k in ("wavelength", "R0", "L", "ncycles", "f_number", "theta", "eps", "P0", "pol_angle",
              "ellipticity", "cep", "gdd", "tod", "bandwidth"):
        setattr(s, k, float(p.get(k, 0.0)))
    bumps = p.get("bumps")
    if bumps is not None and len(bumps):
        arr = (ctypes.c_double * (4 * len(bumps)))(*[float(v) for b in bumps for v in b])
        s._bumps_keepalive = arr               # the struct only points at it
        s.nbumps = len(bumps)
        s.bumps = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    return s


def info_dict(s):
    d = {k: getattr(s, k) for k, _ in tf_pulse_info._fields_ if k != "reserved"}
    d["overlap"] = bool(d["overlap"])
    return d


def window_struct(w):
    if isinstance(w, tf_window):
        return w
    return tf_window(int(w["wx"]), int(w["wy"]), int(w["wz"]), 0,
                     float(w["cx"]), float(w["cy"]), float(w["cz"]))


def _buffer(a):
    """(pointer, on_device, nbytes, itemsize) of a torch tensor or numpy array."""
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), 1 if a.is_cuda else 0, a.numel() * a.element_size(), a.element_size()
    import numpy as np
    if not (isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"]):
        raise ValueError("need a C-contiguous numpy array or a contiguous tensor")
    return a.ctypes.data, 0, a.nbytes, a.itemsize


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ---- C calls ------------------------------------------------------------------

def tf_version():
    return load().tf_version().decode()


def tf_last_error():
    return load().tf_last_error().decode()


def tf_supported_length(n):
    return bool(load().tf_supported_length(int(n)))


def tf_pulse_geometry(pulse):
    info = tf_pulse_info()
    _check(load().tf_pulse_geometry(ctypes.byref(pulse_struct(pulse)), ctypes.byref(info)))
    return info_dict(info)


def tf_layer_grid(pulse, n, spacing):
    out = tf_grid()
    _check(load().tf_layer_grid(ctypes.byref(pulse_struct(pulse)), int(n[0]), int(n[1]), int(n[2]),
                                float(spacing[0]), float(spacing[1]), float(spacing[2]),
                                ctypes.byref(out)))
    return grid_dict(out)


def tf_create(grid, precision="f32", stream=None):
    h = ctypes.c_void_p()
    prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
    _check(load().tf_create(ctypes.byref(grid_struct(grid)), prec, _stream_ptr(stream), ctypes.byref(h)))
    return h


def tf_destroy(h):
    _check(load().tf_destroy(h))


def tf_set_fields(h, src, t=0.0):
    ptr, dev, _, _ = _buffer(src)
    _check(load().tf_set_fields(h, ptr, dev, float(t)))


def tf_get_fields(h, dst):
    ptr, dev, _, _ = _buffer(dst)
    _check(load().tf_get_fields(h, ptr, dev))
    return dst


def tf_state_ptr(h):
    p = ctypes.c_void_p()
    _check(load().tf_state_ptr(h, ctypes.byref(p)))
    return p.value


def tf_set_pulse(h, pulse):
    info = tf_pulse_info()
    _check(load().tf_set_pulse(h, ctypes.byref(pulse_struct(pulse)), ctypes.byref(info)))
    return info_dict(info)


def tf_set_cutout(h, R_min, R_max):
    _check(load().tf_set_cutout(h, float(R_min), float(R_max)))


def tf_advance(h, nsteps, dt):
    _check(load().tf_advance(h, int(nsteps), float(dt)))


def tf_advance_current(h, j, dt):
    """One step of dt with the current density j (3 x nz x ny x nx of the
    solver's precision, host array or device tensor) held over the step."""
    ptr, dev, _, _ = _buffer(j)
    _check(load().tf_advance_current(h, ctypes.c_void_p(ptr), dev, float(dt)))


def tf_read_focal(h, window, dst):
    ptr, dev, _, _ = _buffer(dst)
    _check(load().tf_read_focal(h, ctypes.byref(window_struct(window)), ptr, dev))
    return dst


def tf_diagnostics(h):
    e, de, db = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().tf_diagnostics(h, ctypes.byref(e), ctypes.byref(de), ctypes.byref(db)))
    return e.value, de.value, db.value


def tf_advance_diagnosed(h, nsteps, dt):
    """nsteps steps of dt; (energy, max_div_e, max_div_b) of the new state
    from the last step's z pass."""
    e, de, db = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().tf_advance_diagnosed(h, int(nsteps), float(dt), ctypes.byref(e), ctypes.byref(de),
                                       ctypes.byref(db)))
    return e.value, de.value, db.value


def tf_time(h):
    t = ctypes.c_double()
    _check(load().tf_time(h, ctypes.byref(t)))
    return t.value


def tf_get_grid(h):
    g = tf_grid()
    _check(load().tf_get_grid(h, ctypes.byref(g)))
    return grid_dict(g)


def tf_profile(h, enable):
    _check(load().tf_profile(h, 1 if enable else 0))


def tf_profile_read(h):
    """{pass name: (total ms, launches)} since profiling was enabled."""
    ms = (ctypes.c_double * len(PASS_NAMES))()
    n = (ctypes.c_int64 * len(PASS_NAMES))()
    _check(load().tf_profile_read(h, ms, n))
    return {k: (ms[i], n[i]) for i, k in enumerate(PASS_NAMES)}


def tf_set_plan_file(path):
    _check(load().tf_set_plan_file(path.encode() if path else None))


def tf_advance_noalloc(grid, precision, state, nsteps, dt, project_b_first=False, stream=None):
    """Advance a device state [6][nz][ny][nx] in place without allocating."""
    ptr, dev, nbytes, isz = _buffer(state)
    if not dev:
        raise ValueError("tf_advance_noalloc needs a device state")
    prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
    g = grid_struct(grid)
    if isz != (8 if prec == TF_F64 else 4) or nbytes != 6 * g.nx * g.ny * g.nz * isz:
        raise ValueError("state must hold 6 nx ny nz elements of the precision's type")
    _check(load().tf_advance_noalloc(ctypes.byref(g), prec, ctypes.c_void_p(ptr), int(nsteps),
                                     float(dt), 1 if project_b_first else 0, _stream_ptr(stream)))


def tf_kernel_plan(grid, precision="f32"):
    """(row_block, fast, zvariant, ystrip) that tf_create would use for the grid."""
    rb, fast, zv, ys = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
    _check(load().tf_kernel_plan(ctypes.byref(grid_struct(grid)), prec, ctypes.byref(rb), ctypes.byref(fast),
                                 ctypes.byref(zv), ctypes.byref(ys)))
    return rb.value, bool(fast.value), zv.value, ys.value


def tf_tune(sizes, precision, plan_path):
    """Tune the kernel plans of the cube sizes; returns best ms per step."""
    arr = (ctypes.c_int32 * len(sizes))(*sizes)
    best = (ctypes.c_double * len(sizes))()
    prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
    _check(load().tf_tune(arr, len(sizes), prec, plan_path.encode(), best))
    return list(best)


class Batch:
    """Owning wrapper of a tf_batch (uneven-grid parameter sweep)."""

    def __init__(self, grids, pulses, precision="f32", stream=None):
        if len(grids) != len(pulses) or not grids:
            raise ValueError("need equal, non-empty lists of grids and pulses")
        self.n = len(grids)
        self.precision = precision
        self.itemsize = 8 if precision == "f64" else 4
        self.grids = [grid_dict(grid_struct(g)) for g in grids]
        G = (tf_grid * self.n)(*[grid_struct(g) for g in grids])
        P = (tf_pulse * self.n)(*[pulse_struct(p) for p in pulses])
        h = ctypes.c_void_p()
        prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
        _check(load().tf_batch_create(G, P, self.n, prec, _stream_ptr(stream), ctypes.byref(h)))
        self.h = h
        self._ran = False

    def close(self):
        if self.h is not None and self.h.value:
            _check(load().tf_batch_destroy(self.h))
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, nsteps, dt, window, dst, use_graph=True):
        """dst: device tensor holding n x 6 x wz x wy x wx elements."""
        if len(nsteps) != self.n or len(dt) != self.n:
            raise ValueError("need one nsteps and one dt per instance")
        w = window_struct(window)
        ptr, dev, nbytes, item = _buffer(dst)
        if not dev:
            raise ValueError("batch windows are written to device memory")
        if item != self.itemsize or nbytes != self.n * 6 * w.wx * w.wy * w.wz * item:
            raise ValueError("dst must hold n x 6 x wz x wy x wx elements of the batch precision")
        ns = (ctypes.c_int64 * self.n)(*[int(v) for v in nsteps])
        ds = (ctypes.c_double * self.n)(*[float(v) for v in dt])
        _check(load().tf_batch_run(self.h, ns, ds, ctypes.byref(w), ptr, 1 if use_graph else 0))
        self._ran = True

    def get_fields(self, i, dst):
        g = self.grids[i]
        ptr, dev, nbytes, item = _buffer(dst)
        if item != self.itemsize or nbytes != 6 * g["nx"] * g["ny"] * g["nz"] * item:
            raise ValueError("dst must hold the instance state")
        _check(load().tf_batch_get_fields(self.h, int(i), ptr, dev))
        return dst


class Solver:
    """Owning wrapper of a tf_solver handle; checks buffer sizes and element
    types before passing pointers to the library."""

    def __init__(self, grid, precision="f32", stream=None):
        self.precision = precision
        self.itemsize = 8 if precision == "f64" else 4
        self.grid = grid_dict(grid_struct(grid))
        self.h = tf_create(grid, precision, stream)

    def close(self):
        if self.h is not None and self.h.value:
            tf_destroy(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        g = self.grid
        return (6, g["nz"], g["ny"], g["nx"])

    def _expect(self, a, shape):
        _, _, nbytes, item = _buffer(a)
        n = 1
        for v in shape:
            n *= v
        if item != self.itemsize or nbytes != n * self.itemsize:
            raise ValueError(f"buffer must hold {shape} elements of {self.itemsize} bytes")

    def set_fields(self, src, t=0.0):
        self._expect(src, self.shape)
        tf_set_fields(self.h, src, t)

    def get_fields(self, dst):
        self._expect(dst, self.shape)
        return tf_get_fields(self.h, dst)

    def set_pulse(self, pulse):
        return tf_set_pulse(self.h, pulse)

    def set_cutout(self, R_min, R_max):
        tf_set_cutout(self.h, R_min, R_max)

    def advance(self, nsteps, dt):
        tf_advance(self.h, nsteps, dt)

    def advance_current(self, j, dt):
        """One step of dt with the current density j held over the step."""
        self._expect(j, (3,) + tuple(self.shape[1:]))
        tf_advance_current(self.h, j, dt)

    def read_focal(self, window, dst):
        w = window_struct(window)
        self._expect(dst, (6, w.wz, w.wy, w.wx))
        return tf_read_focal(self.h, w, dst)

    def diagnostics(self):
        return tf_diagnostics(self.h)

    def advance_diagnosed(self, nsteps, dt):
        return tf_advance_diagnosed(self.h, nsteps, dt)

    @property
    def t(self):
        return tf_time(self.h)

    def state_ptr(self):
        return tf_state_ptr(self.h)

    def profile(self, enable=True):
        tf_profile(self.h, enable)

    def profile_read(self):
        return tf_profile_read(self.h)


# ---- learned surrogate ----------------------------------------------------------

FNO_N, FNO_WIDTH, FNO_MODES, FNO_NPARAM, FNO_HIDDEN, FNO_NOUT, FNO_LAYERS = 64, 32, 12, 8, 128, 6, 3
FNO_NMODES = 4 * FNO_MODES ** 3


def fno_param_shapes(nbasis=1):
    """(name, shape) of the flat parameter vector in order for a head of
    nbasis basis fields; R entries are complex (stored as re, im pairs)."""
    C, H = FNO_WIDTH, FNO_HIDDEN
    out = [("W0", (FNO_NPARAM + 3, C)), ("b0", (C,))]
    for l in range(1, FNO_LAYERS + 1):
        out += [(f"W{l}", (C, C)), (f"b{l}", (C,)), (f"R{l}", (FNO_NMODES, C, C))]
    out += [("P1", (C, H)), ("c1", (H,)), ("P2", (H, FNO_NOUT * nbasis)), ("c2", (FNO_NOUT * nbasis,))]
    return out


def fno_flatten(params):
    """dict of numpy arrays (R complex) -> flat float32 vector."""
    import numpy as np
    nbasis = np.shape(params["P2"])[1] // FNO_NOUT
    parts = []
    for name, shape in fno_param_shapes(nbasis):
        a = np.asarray(params[name])
        if a.shape != shape:
            raise ValueError(f"{name} must have shape {shape}")
        if name.startswith("R"):
            a = np.stack([a.real, a.imag], axis=-1)
        parts.append(np.ascontiguousarray(a, dtype=np.float32).ravel())
    flat = np.concatenate(parts)
    assert flat.size == load().tf_fno_param_count(nbasis)
    return flat


def fno_unflatten(flat):
    """flat vector -> dict of float64 arrays (R complex128)."""
    import numpy as np
    flat = np.asarray(flat, dtype=np.float64)
    nbasis = [k for k in (1, 2, 4) if load().tf_fno_param_count(k) == flat.size]
    if not nbasis:
        raise ValueError("not a surrogate parameter vector")
    out, o = {}, 0
    for name, shape in fno_param_shapes(nbasis[0]):
        n = int(np.prod(shape)) * (2 if name.startswith("R") else 1)
        a = flat[o:o + n]
        o += n
        out[name] = (a[0::2] + 1j * a[1::2]).reshape(shape) if name.startswith("R") else a.reshape(shape)
    return out


def tf_fno_phasor_weights(pulse, nbasis):
    """Head weights of a pulse (numpy float64 array of nbasis entries)."""
    import numpy as np
    w = (ctypes.c_double * 4)()
    _check(load().tf_fno_phasor_weights(ctypes.byref(pulse_struct(pulse)), int(nbasis), w))
    return np.array(w[:nbasis])


class Surrogate:
    """Owning wrapper of a tf_fno (Fourier neural operator surrogate).
    params, head weights, targets and outputs are contiguous float32 CUDA
    tensors."""

    def __init__(self, max_batch, training=False, nbasis=1, stream=None, period=FNO_N):
        h = ctypes.c_void_p()
        _check(load().tf_fno_create(int(max_batch), 1 if training else 0, int(nbasis), _stream_ptr(stream),
                                    ctypes.byref(h)))
        self.h = h
        self.max_batch = int(max_batch)
        self.training = bool(training)
        self.nbasis = int(nbasis)
        self.nparams = int(load().tf_fno_param_count(self.nbasis))
        if period != FNO_N:
            self.set_period(period)

    def set_period(self, period):
        """Period of the spectral transform (64: plain; > 64: zero-padded)."""
        _check(load().tf_fno_set_period(self.h, int(period)))

    @property
    def period(self):
        p = ctypes.c_int32()
        _check(load().tf_fno_get_period(self.h, ctypes.byref(p)))
        return p.value

    def close(self):
        if self.h is not None and self.h.value:
            _check(load().tf_fno_destroy(self.h))
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dev(t, shape, what):
        ptr, dev, nbytes, item = _buffer(t)
        n = 1
        for v in shape:
            n *= v
        if not dev or item != 4 or nbytes != 4 * n:
            raise ValueError(f"{what} must be a float32 device tensor of shape {shape}")
        return ptr

    def set_params(self, params):
        """dict (oracle layout) or flat float32 array/tensor."""
        flat = fno_flatten(params) if isinstance(params, dict) else params
        ptr, dev, nbytes, item = _buffer(flat)
        if item != 4 or nbytes != 4 * self.nparams:
            raise ValueError("flat parameters must be float32 of tf_fno_param_count() entries")
        _check(load().tf_fno_set_params(self.h, ptr, dev))

    def get_params(self):
        import numpy as np
        flat = np.empty(self.nparams, np.float32)
        _check(load().tf_fno_get_params(self.h, flat.ctypes.data, 0))
        return flat

    def _w(self, w, B):
        if w is None:
            if self.nbasis != 1:
                raise ValueError("this head needs per-sample weights")
            return None
        return self._dev(w, (B, self.nbasis), "head weights")

    def forward(self, p, out, w=None, graph=False):
        """out <- surrogate(p) with head weights w; graph=True replays a
        captured hipGraph."""
        B = p.shape[0]
        pp = self._dev(p, (B, FNO_NPARAM), "params")
        po = self._dev(out, (B, FNO_NOUT, FNO_N, FNO_N, FNO_N), "out")
        fn = load().tf_fno_infer if graph else load().tf_fno_forward
        _check(fn(self.h, pp, self._w(w, B), B, po))
        return out

    def loss_grad(self, p, target, w=None, want_grad=True):
        import numpy as np
        B = p.shape[0]
        pp = self._dev(p, (B, FNO_NPARAM), "params")
        pt = self._dev(target, (B, FNO_NOUT, FNO_N, FNO_N, FNO_N), "target")
        loss = ctypes.c_double()
        g = np.empty(self.nparams, np.float32) if want_grad else None
        _check(load().tf_fno_loss_grad(self.h, pp, self._w(w, B), pt, B, ctypes.byref(loss),
                                        g.ctypes.data if want_grad else None))
        return loss.value, g

    def train_step(self, p, target, lr, w=None, want_loss=True):
        B = p.shape[0]
        pp = self._dev(p, (B, FNO_NPARAM), "params")
        pt = self._dev(target, (B, FNO_NOUT, FNO_N, FNO_N, FNO_N), "target")
        loss = ctypes.c_double()
        _check(load().tf_fno_train_step(self.h, pp, self._w(w, B), pt, B, float(lr),
                                         ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def train(self, p, target, epochs, batch, lr, w=None, lr_min_frac=0.02, seed=0, scale_targets=True,
              progress=None):
        """tf_fno_train over n samples (device tensors p [n, 8], w [n, K],
        target [n, 6, 64, 64, 64]); returns the per-epoch mean losses.
        progress(epoch, loss), if given, is called after every epoch."""
        import numpy as np
        n = p.shape[0]
        pp = self._dev(p, (n, FNO_NPARAM), "params")
        pt = self._dev(target, (n, FNO_NOUT, FNO_N, FNO_N, FNO_N), "target")
        pw = None
        if self.nbasis != 1:
            pw = self._dev(w, (n, self.nbasis), "head weights")
        hist = np.zeros(int(epochs), dtype=np.float64)
        cb = TRAIN_PROGRESS(lambda ep, loss, _u: progress(int(ep), float(loss))) if progress else TRAIN_PROGRESS()
        cfg = tf_train_cfg(int(epochs), int(batch), float(lr), float(lr_min_frac), int(seed),
                           1 if scale_targets else 0, 0, hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           cb, None)
        last = ctypes.c_double()
        _check(load().tf_fno_train(self.h, pp, pw, pt, int(n), ctypes.byref(cfg), ctypes.byref(last)))
        return hist

    def eval(self, p, target, w=None):
        """tf_fno_eval: per-sample relative L2 error (numpy array)."""
        import numpy as np
        n = p.shape[0]
        pp = self._dev(p, (n, FNO_NPARAM), "params")
        pt = self._dev(target, (n, FNO_NOUT, FNO_N, FNO_N, FNO_N), "target")
        pw = None
        if self.nbasis != 1:
            pw = self._dev(w, (n, self.nbasis), "head weights")
        out = np.zeros(int(n), dtype=np.float64)
        _check(load().tf_fno_eval(self.h, pp, pw, pt, int(n), out.ctypes.data))
        return out

    def spectral_forward(self, v, modes):
        B = v.shape[0]
        pv = self._dev(v, (B, FNO_N, FNO_N, FNO_N, FNO_WIDTH), "v")
        pm = self._dev(modes, (B, 2 * FNO_MODES, 2, 2 * FNO_MODES, FNO_MODES, FNO_WIDTH), "modes")
        _check(load().tf_fno_spectral_forward(self.h, pv, B, pm))
        return modes

    def spectral_inverse(self, modes, u):
        B = u.shape[0]
        pm = self._dev(modes, (B, 2 * FNO_MODES, 2, 2 * FNO_MODES, FNO_MODES, FNO_WIDTH), "modes")
        pu = self._dev(u, (B, FNO_N, FNO_N, FNO_N, FNO_WIDTH), "u")
        _check(load().tf_fno_spectral_inverse(self.h, pm, B, pu))
        return u

    def save(self, path):
        _check(load().tf_fno_save(self.h, str(path).encode()))

    def load_checkpoint(self, path):
        _check(load().tf_fno_load(self.h, str(path).encode()))
