"""Python binding of the MI355X AIREBO library (``libairebo.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/airebo.h``.  Device memory and
the stream come from PyTorch.  There is no CPU fallback: if the library is
missing or no GPU is visible, the calls raise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libairebo.so")
DEFAULT_PARAMS = os.path.join(HERE, "params", "airebo_ch.param")

FP64, MIXED, SINGLE = 0, 1, 2
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "single": SINGLE}
VDW_LJ, VDW_MORSE = 0, 1
TERM_REBO, TERM_LJ, TERM_TORSION, TERM_ALL = 1, 2, 4, 7
THERMO_COLUMNS = ("step", "PE", "KE", "Etot", "T", "rebuilds", "P_bar")
STAT_NAMES = ["lj_in_cut", "cij_zero", "bstar_queued", "dsb_nonzero", "bonds", "rebuilds", "max_short",
              "lj_entries", "max_lj", "spline_evals", "spline_evals_fp64", "nn_fallbacks",
              "regrowths", "slow_path_pairs", "deferred_pairs", "lj_in_cut_far", "lj_entries_far", "max_lj_far"]

EXPORTS = ["airebo_options_default", "airebo_ctx_create", "airebo_ctx_free", "airebo_compute", "airebo_nve",
           "airebo_stats", "airebo_stats_n", "airebo_last_error", "airebo_profile_nve", "airebo_kernel_count", "airebo_kernel_name",
           "airebo_batch_compute", "airebo_batch_nve",
           "airebo_nn_create", "airebo_nn_free", "airebo_nn_sizes", "airebo_nn_models", "airebo_nn_set_params",
           "airebo_nn_get_params", "airebo_nn_get_grad", "airebo_nn_set_norm", "airebo_nn_get_norm",
           "airebo_nn_moments", "airebo_nn_descriptors", "airebo_nn_descriptor_jvp", "airebo_nn_descriptor_vjp",
           "airebo_nn_compute", "airebo_nn_gradient", "airebo_nn_adam", "airebo_nn_nve", "airebo_nn_profile_nve",
           "airebo_nn_save", "airebo_nn_load", "airebo_nn_mfma_check", "airebo_nn_mfma32_check", "airebo_peak_copy", "airebo_peak_fma",
           "airebo_params_load", "airebo_params_parse", "airebo_params_free", "airebo_ctx_create_from_params",
           "airebo_compute_host", "airebo_nn_train_step",
           "airebo_md_begin", "airebo_batch_md_begin", "airebo_md_run", "airebo_md_state", "airebo_md_end",
           "airebo_nn_md_begin", "airebo_compute_static"]


class AireboError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"airebo error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("term_mask", ctypes.c_int32), ("skin", ctypes.c_double),
                ("lj_cap", ctypes.c_int32), ("device", ctypes.c_int32), ("bond_block", ctypes.c_int32),
                ("bond_grid", ctypes.c_int32), ("defer_block", ctypes.c_int32), ("short_block", ctypes.c_int32),
                ("vdw", ctypes.c_int32), ("lj_slack", ctypes.c_int32), ("queue_per_atom", ctypes.c_int32),
                ("schedule", ctypes.c_int32)]

    TUNABLES = ("bond_block", "bond_grid", "defer_block", "short_block", "schedule")
    CAPACITIES = ("lj_slack", "queue_per_atom")


_lib = None


def load_library(path=LIB_PATH):
    """Load libairebo.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise AireboError(-1, f"{path} is not built; run python -m paper_1810_07026_amd.build")
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
    L.airebo_options_default.argtypes = [ctypes.POINTER(Options)]
    L.airebo_options_default.restype = None
    L.airebo_ctx_create.argtypes = [ctypes.c_char_p, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]
    L.airebo_ctx_create.restype = ctypes.c_int
    L.airebo_params_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
    L.airebo_params_load.restype = ctypes.c_int
    L.airebo_params_parse.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
    L.airebo_params_parse.restype = ctypes.c_int
    L.airebo_params_free.argtypes = [vp]
    L.airebo_params_free.restype = None
    L.airebo_ctx_create_from_params.argtypes = [vp, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]
    L.airebo_ctx_create_from_params.restype = ctypes.c_int
    hdp = ctypes.POINTER(ctypes.c_double)
    L.airebo_compute_host.argtypes = [vp, ctypes.c_int64, hdp, ctypes.POINTER(ctypes.c_int32), hdp,
                                      ctypes.POINTER(ctypes.c_int32), hdp, hdp, hdp]
    L.airebo_compute_host.restype = ctypes.c_int
    L.airebo_compute_static.argtypes = [vp, ctypes.c_int64, dp, ip, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32), dp, dp, dp, vp]
    L.airebo_compute_static.restype = ctypes.c_int
    L.airebo_ctx_free.argtypes = [vp]
    L.airebo_ctx_free.restype = None
    L.airebo_compute.argtypes = [vp, ctypes.c_int64, dp, ip, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int32), dp, dp, dp, vp]
    L.airebo_compute.restype = ctypes.c_int
    L.airebo_nve.argtypes = [vp, ctypes.c_int64, dp, dp, ip, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                             ctypes.c_int64, ctypes.c_int64, dp, vp]
    L.airebo_nve.restype = ctypes.c_int
    L.airebo_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.airebo_stats.restype = ctypes.c_int
    L.airebo_stats_n.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    L.airebo_stats_n.restype = ctypes.c_int
    L.airebo_profile_nve.argtypes = L.airebo_nve.argtypes[:10] + [ctypes.POINTER(ctypes.c_double),
                                                                   ctypes.POINTER(ctypes.c_int64), vp]
    L.airebo_profile_nve.restype = ctypes.c_int
    L.airebo_kernel_count.argtypes = []
    L.airebo_kernel_count.restype = ctypes.c_int
    L.airebo_kernel_name.argtypes = [ctypes.c_int]
    L.airebo_kernel_name.restype = ctypes.c_char_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.airebo_batch_compute.argtypes = [vp, ctypes.c_int32, i64p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32), dp, ip, dp, dp, dp, vp]
    L.airebo_batch_compute.restype = ctypes.c_int
    L.airebo_batch_nve.argtypes = [vp, ctypes.c_int32, i64p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int32), dp, dp, ip, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_double, ctypes.c_int64, ctypes.c_int64, dp, vp]
    L.airebo_batch_nve.restype = ctypes.c_int
    hdp2 = ctypes.POINTER(ctypes.c_double)
    L.airebo_md_begin.argtypes = [vp, ctypes.c_int64, dp, dp, ip, hdp2, ctypes.POINTER(ctypes.c_int32), hdp2,
                                  ctypes.c_double, vp]
    L.airebo_md_begin.restype = ctypes.c_int
    L.airebo_batch_md_begin.argtypes = [vp, ctypes.c_int32, i64p, hdp2, ctypes.POINTER(ctypes.c_int32), dp, dp, ip,
                                        hdp2, ctypes.c_double, vp]
    L.airebo_batch_md_begin.restype = ctypes.c_int
    L.airebo_md_run.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, dp, vp]
    L.airebo_md_run.restype = ctypes.c_int
    L.airebo_md_state.argtypes = [vp, dp, dp, vp]
    L.airebo_md_state.restype = ctypes.c_int
    L.airebo_md_end.argtypes = [vp]
    L.airebo_md_end.restype = None
    L.airebo_last_error.argtypes = []
    L.airebo_last_error.restype = ctypes.c_char_p
    # learned surrogate
    c_d, c_i32, c_i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    hd, hi32 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    geo = [vp, vp, c_i64, dp, ip, hd, hi32]      # nn, ctx, n, pos, species, box, periodic
    sig = {
        "airebo_nn_create": [c_i32, c_i32, ctypes.POINTER(ctypes.c_void_p)],
        "airebo_nn_sizes": [hi32, hi32],
        "airebo_nn_models": [vp],
        "airebo_nn_set_params": [vp, vp],
        "airebo_nn_get_params": [vp, vp],
        "airebo_nn_get_grad": [vp, vp],
        "airebo_nn_set_norm": [vp, vp, vp, c_d, hd],
        "airebo_nn_get_norm": [vp, vp, vp, hd, hd],
        "airebo_nn_moments": [vp, dp, c_i64, hd, vp],
        "airebo_nn_descriptors": geo + [dp, vp],
        "airebo_nn_descriptor_jvp": geo + [dp, dp, vp],
        "airebo_nn_descriptor_vjp": geo + [dp, c_i32, dp, dp, vp],
        "airebo_nn_compute": geo + [c_d, dp, dp, dp, dp, hd, vp],
        "airebo_nn_gradient": geo + [dp, c_d, c_d, c_d, hd, vp],
        "airebo_nn_adam": [vp, c_d, c_d, c_d, c_d, vp],
        "airebo_nn_train_step": geo + [dp, c_d, c_d, c_d, c_d, hd, vp],
        "airebo_nn_nve": [vp, vp, c_i64, dp, dp, ip, hd, hi32, hd, c_d, c_i64, c_i64, dp, c_d,
                          ctypes.POINTER(ctypes.c_int64), vp],
        "airebo_nn_md_begin": [vp, vp, c_i64, dp, dp, ip, hd, hi32, hd, c_d, c_d, vp],
        "airebo_nn_profile_nve": [vp, vp, c_i64, dp, dp, ip, hd, hi32, hd, c_d, c_i64, c_d,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), vp],
        "airebo_nn_save": [vp, ctypes.c_char_p],
        "airebo_nn_load": [ctypes.c_char_p, c_i32, ctypes.POINTER(ctypes.c_void_p)],
        "airebo_nn_mfma_check": [dp, dp, dp, vp],
        "airebo_nn_mfma32_check": [dp, dp, dp, vp],
        "airebo_peak_copy": [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp],
        "airebo_peak_fma": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.airebo_nn_free.argtypes = [vp]
    L.airebo_nn_free.restype = None
    _lib = L
    return L


def _check(L, rc):
    if rc != 0:
        raise AireboError(rc, L.airebo_last_error().decode())


def _host3(a, ctype):
    arr = (ctype * 3)(*a)
    return arr


def _state(t, n, name, device):
    """A positions or velocities tensor the library may read and write as
    double [n][3]: float64, contiguous, shape (n, 3), on the context's device."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device == device):
        raise AireboError(-1, f"{name} must be a CUDA tensor on {device}")
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (n, 3):
        raise AireboError(-1, f"{name} must be a contiguous float64 tensor of shape ({n}, 3), "
                              f"got {t.dtype} {tuple(t.shape)}{'' if t.is_contiguous() else ' (non-contiguous)'}")
    return t


class ParamSet:
    """A validated AIREBO parameter set held on the host (airebo_params_*):
    from a file path, or from the file's text with text=..."""

    def __init__(self, path=DEFAULT_PARAMS, text=None):
        self.L = load_library()
        h = ctypes.c_void_p()
        if text is not None:
            b = text.encode() if isinstance(text, str) else bytes(text)
            _check(self.L, self.L.airebo_params_parse(b, len(b), ctypes.byref(h)))
        else:
            _check(self.L, self.L.airebo_params_load(path.encode(), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.airebo_params_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Context:
    """One AIREBO evaluation context on one GPU (params: a file path or a ParamSet)."""

    def __init__(self, params=DEFAULT_PARAMS, precision=FP64, term_mask=TERM_ALL, skin=1.0, lj_cap=0, device=0,
                 tune=None, vdw=VDW_LJ):
        import torch
        if not torch.cuda.is_available():
            raise AireboError(-7, "no GPU visible: the AIREBO library runs on the GPU only")
        self.L = load_library()
        o = Options()
        self.L.airebo_options_default(ctypes.byref(o))
        o.precision, o.term_mask, o.skin, o.lj_cap, o.device = precision, term_mask, skin, lj_cap, device
        o.vdw = vdw
        for k, v in (tune or {}).items():
            if k not in Options.TUNABLES + Options.CAPACITIES:
                raise AireboError(-1, f"unknown tunable {k}")
            setattr(o, k, int(v))
        self.tune = dict(tune or {})
        h = ctypes.c_void_p()
        if isinstance(params, ParamSet):
            _check(self.L, self.L.airebo_ctx_create_from_params(params.h, ctypes.byref(o), ctypes.byref(h)))
        else:
            _check(self.L, self.L.airebo_ctx_create(params.encode(), ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if getattr(self, "h", None):
            self.L.airebo_ctx_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, a, dtype):
        import torch
        t = torch.as_tensor(a, dtype=dtype, device=self.device)
        return t.contiguous()

    def compute_host(self, x, species, box, periodic=(1, 1, 1)):
        """airebo_compute on host (numpy) arrays: energy [4], forces [n,3], virial [6] as numpy arrays."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        s = np.ascontiguousarray(species, dtype=np.int32)
        n = len(s)
        e, w, f = np.zeros(4), np.zeros(6), np.zeros((n, 3))
        dpp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(self.L, self.L.airebo_compute_host(self.h, n, dpp(x), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                  _host3(box, ctypes.c_double), _host3(periodic, ctypes.c_int32),
                                                  dpp(e), dpp(f), dpp(w)))
        return e, f, w

    def compute(self, x, species, box, periodic=(1, 1, 1), out=None):
        """Energy [4] (total, REBO, LJ, torsion), forces [n,3], virial [6] as device tensors."""
        import torch
        x = self._dev(x, torch.float64).reshape(-1, 3)
        s = self._dev(species, torch.int32)
        n = x.shape[0]
        e = torch.empty(4, dtype=torch.float64, device=self.device)
        w = torch.empty(6, dtype=torch.float64, device=self.device)
        f = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device=self.device)
        rc = self.L.airebo_compute(self.h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                   _host3(box, ctypes.c_double), _host3(periodic, ctypes.c_int32),
                                   ctypes.c_void_p(e.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                   ctypes.c_void_p(w.data_ptr()), self._stream())
        _check(self.L, rc)
        return e, f, w

    def compute_static(self, x, species, box, periodic=(1, 1, 1), energy=None, forces=None, virial=None):
        """airebo_compute_static (no device allocation inside the library): energy [4], forces [n,3],
        virial [6] as device tensors; pass preallocated outputs to allocate nothing here either."""
        import torch
        x = self._dev(x, torch.float64).reshape(-1, 3)
        s = self._dev(species, torch.int32)
        n = x.shape[0]
        e = energy if energy is not None else torch.empty(4, dtype=torch.float64, device=self.device)
        w = virial if virial is not None else torch.empty(6, dtype=torch.float64, device=self.device)
        f = forces if forces is not None else torch.empty((n, 3), dtype=torch.float64, device=self.device)
        for t, shape in ((e, (4,)), (w, (6,)), (f, (n, 3))):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape or t.device != self.device:
                raise AireboError(-1, f"output must be a contiguous float64 tensor of shape {shape} on {self.device}")
        rc = self.L.airebo_compute_static(self.h, n, _p(x), _p(s), _host3(box, ctypes.c_double),
                                          _host3(periodic, ctypes.c_int32), _p(e), _p(f), _p(w), self._stream())
        _check(self.L, rc)
        return e, f, w

    def nve(self, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5, nsteps=10,
            thermo_every=1):
        """Velocity Verlet in place on device tensors x, v; returns the thermo rows (device tensor,
        columns THERMO_COLUMNS)."""
        import torch
        s = self._dev(species, torch.int32)
        n = s.shape[0]
        _state(x, n, "x", self.device)
        _state(v, n, "v", self.device)
        rows = nsteps // thermo_every + 1 if thermo_every > 0 else 1
        th = torch.zeros((rows, len(THERMO_COLUMNS)), dtype=torch.float64, device=self.device)
        m = (ctypes.c_double * 2)(*masses)
        rc = self.L.airebo_nve(self.h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                               ctypes.c_void_p(s.data_ptr()), _host3(box, ctypes.c_double),
                               _host3(periodic, ctypes.c_int32), m, dt, nsteps, thermo_every,
                               ctypes.c_void_p(th.data_ptr()), self._stream())
        _check(self.L, rc)
        return th

    def profile_nve(self, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5, nsteps=10):
        """Per-kernel device time over nsteps eager NVE steps: {name: (total ms, launches)}."""
        import torch
        s = self._dev(species, torch.int32)
        _state(x, s.shape[0], "x", self.device)
        _state(v, s.shape[0], "v", self.device)
        nk = self.L.airebo_kernel_count()
        ms = (ctypes.c_double * nk)()
        cnt = (ctypes.c_int64 * nk)()
        m = (ctypes.c_double * 2)(*masses)
        rc = self.L.airebo_profile_nve(self.h, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                       _host3(box, ctypes.c_double), _host3(periodic, ctypes.c_int32), m, dt,
                                       nsteps, ms, cnt, self._stream())
        _check(self.L, rc)
        return {self.L.airebo_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(nk)}

    @staticmethod
    def _batch_host(sizes, boxes, periodic):
        nsys = len(sizes)
        off = np.zeros(nsys + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        b = np.ascontiguousarray(boxes, dtype=np.float64).reshape(nsys, 3)
        p = np.ascontiguousarray(periodic if periodic is not None else np.ones((nsys, 3)), dtype=np.int32)
        p = np.ascontiguousarray(np.broadcast_to(p.reshape(-1, 3), (nsys, 3)), dtype=np.int32)
        return nsys, off, b, p

    def batch_compute(self, x, species, sizes, boxes, periodic=None):
        """Batched evaluation: energy [nsys,4], forces [n,3], virial [nsys,6] (device tensors)."""
        import torch
        x = self._dev(x, torch.float64).reshape(-1, 3)
        s = self._dev(species, torch.int32)
        nsys, off, b, p = self._batch_host(sizes, boxes, periodic)
        e = torch.empty((nsys, 4), dtype=torch.float64, device=self.device)
        w = torch.empty((nsys, 6), dtype=torch.float64, device=self.device)
        f = torch.empty((x.shape[0], 3), dtype=torch.float64, device=self.device)
        rc = self.L.airebo_batch_compute(
            self.h, nsys, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(e.data_ptr()),
            ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(w.data_ptr()), self._stream())
        _check(self.L, rc)
        return e, f, w

    def batch_nve(self, x, v, species, sizes, boxes, periodic=None, masses=(12.011, 1.008), dt=0.5, nsteps=10,
                  thermo_every=1):
        """Batched velocity Verlet in place; returns thermo [rows, nsys, 7] (device tensor)."""
        import torch
        s = self._dev(species, torch.int32)
        nsys, off, b, p = self._batch_host(sizes, boxes, periodic)
        if int(off[-1]) != s.shape[0]:
            raise AireboError(-1, f"system sizes add up to {int(off[-1])} atoms, species has {s.shape[0]}")
        _state(x, s.shape[0], "x", self.device)
        _state(v, s.shape[0], "v", self.device)
        rows = nsteps // thermo_every + 1 if thermo_every > 0 else 1
        th = torch.zeros((rows, nsys, len(THERMO_COLUMNS)), dtype=torch.float64, device=self.device)
        m = (ctypes.c_double * 2)(*masses)
        rc = self.L.airebo_batch_nve(
            self.h, nsys, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(s.data_ptr()), m, dt,
            nsteps, thermo_every, ctypes.c_void_p(th.data_ptr()), self._stream())
        _check(self.L, rc)
        return th

    # ---- MD session: state held on the device between calls
    def md_begin(self, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5):
        """Start an MD session from device tensors x, v (copied; they are not modified)."""
        import torch
        s = self._dev(species, torch.int32)
        n = s.shape[0]
        _state(x, n, "x", self.device)
        _state(v, n, "v", self.device)
        self._md = (n, 1, s)   # the species tensor must outlive the call only; kept for md_state shapes
        m = (ctypes.c_double * 2)(*masses)
        _check(self.L, self.L.airebo_md_begin(self.h, n, _p(x), _p(v), _p(s), _host3(box, ctypes.c_double),
                                              _host3(periodic, ctypes.c_int32), m, dt, self._stream()))

    def batch_md_begin(self, x, v, species, sizes, boxes, periodic=None, masses=(12.011, 1.008), dt=0.5):
        import torch
        s = self._dev(species, torch.int32)
        nsys, off, b, p = self._batch_host(sizes, boxes, periodic)
        if int(off[-1]) != s.shape[0]:
            raise AireboError(-1, f"system sizes add up to {int(off[-1])} atoms, species has {s.shape[0]}")
        _state(x, s.shape[0], "x", self.device)
        _state(v, s.shape[0], "v", self.device)
        self._md = (s.shape[0], nsys, s)
        m = (ctypes.c_double * 2)(*masses)
        _check(self.L, self.L.airebo_batch_md_begin(
            self.h, nsys, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            _p(x), _p(v), _p(s), m, dt, self._stream()))

    def md_run(self, nsteps, thermo_every=0):
        """Advance the session; returns thermo rows [rows, 7] ([rows, nsys, 7] for a batch) or None."""
        import torch
        if getattr(self, "_md", None) is None:
            raise AireboError(-1, "no MD session")
        n, nsys, _ = self._md
        th = None
        if thermo_every > 0:
            rows = nsteps // thermo_every + 1
            shape = (rows, len(THERMO_COLUMNS)) if nsys == 1 else (rows, nsys, len(THERMO_COLUMNS))
            th = torch.zeros(shape, dtype=torch.float64, device=self.device)
        _check(self.L, self.L.airebo_md_run(self.h, nsteps, thermo_every, _p(th) if th is not None else None,
                                            self._stream()))
        return th

    def md_state(self, x=None, v=None):
        """Current positions and velocities of the session (new tensors unless given)."""
        import torch
        if getattr(self, "_md", None) is None:
            raise AireboError(-1, "no MD session")
        n = self._md[0]
        x = torch.empty((n, 3), dtype=torch.float64, device=self.device) if x is None else _state(x, n, "x",
                                                                                                  self.device)
        v = torch.empty((n, 3), dtype=torch.float64, device=self.device) if v is None else _state(v, n, "v",
                                                                                                  self.device)
        _check(self.L, self.L.airebo_md_state(self.h, _p(x), _p(v), self._stream()))
        return x, v

    def md_end(self):
        self.L.airebo_md_end(self.h)
        self._md = None
        self._md_nn = None

    def stats(self):
        out = (ctypes.c_int64 * len(STAT_NAMES))()
        rc = self.L.airebo_stats_n(self.h, out, len(STAT_NAMES))
        if rc < 0:
            _check(self.L, rc)
        return dict(zip(STAT_NAMES, list(out)))


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


class Surrogate:
    """Ensemble of descriptor networks (learned surrogate of the potential).

    Every evaluation takes an AIREBO Context on the same device: its
    neighbour lists, its integrator, and its AIREBO evaluation as the
    fallback when the ensemble disagrees."""

    def __init__(self, nmodels=4, device=0, path=None):
        import torch
        if not torch.cuda.is_available():
            raise AireboError(-7, "no GPU visible: the surrogate runs on the GPU only")
        self.L = load_library()
        h = ctypes.c_void_p()
        if path is not None:
            _check(self.L, self.L.airebo_nn_load(path.encode(), device, ctypes.byref(h)))
        else:
            _check(self.L, self.L.airebo_nn_create(nmodels, device, ctypes.byref(h)))
        self.h = h
        self.device = torch.device("cuda", device)
        d, npar = ctypes.c_int32(), ctypes.c_int32()
        _check(self.L, self.L.airebo_nn_sizes(ctypes.byref(d), ctypes.byref(npar)))
        self.dim, self.npar = d.value, npar.value
        self.nmodels = self.L.airebo_nn_models(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.airebo_nn_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _geo(self, ctx, x, species, box, periodic):
        import torch
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).reshape(-1, 3).contiguous()
        s = torch.as_tensor(species, dtype=torch.int32, device=self.device).contiguous()
        return x, s, [self.h, ctx.h, x.shape[0], _p(x), _p(s), _host3(box, ctypes.c_double),
                      _host3(periodic, ctypes.c_int32)]

    # ---- weights and normalisation
    def set_params(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(self.nmodels, 2, self.npar)
        _check(self.L, self.L.airebo_nn_set_params(self.h, w.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        w = np.zeros((self.nmodels, 2, self.npar), np.float32)
        _check(self.L, self.L.airebo_nn_get_params(self.h, w.ctypes.data_as(ctypes.c_void_p)))
        return w

    def get_grad(self):
        g = np.zeros((self.nmodels, 2, self.npar), np.float32)
        _check(self.L, self.L.airebo_nn_get_grad(self.h, g.ctypes.data_as(ctypes.c_void_p)))
        return g

    def set_norm(self, mean, istd, scale, shift):
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        istd = np.ascontiguousarray(istd, dtype=np.float32)
        sh = (ctypes.c_double * 2)(*shift)
        _check(self.L, self.L.airebo_nn_set_norm(self.h, mean.ctypes.data_as(ctypes.c_void_p),
                                                  istd.ctypes.data_as(ctypes.c_void_p), float(scale), sh))

    def get_norm(self):
        mean = np.zeros(self.dim, np.float32)
        istd = np.zeros(self.dim, np.float32)
        sc = ctypes.c_double()
        sh = (ctypes.c_double * 2)()
        _check(self.L, self.L.airebo_nn_get_norm(self.h, mean.ctypes.data_as(ctypes.c_void_p),
                                                  istd.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sc), sh))
        return mean, istd, sc.value, [sh[0], sh[1]]

    def moments(self, G):
        """Column sums and sums of squares of a device descriptor array [rows, dim]."""
        mom = np.zeros(2 * self.dim)
        _check(self.L, self.L.airebo_nn_moments(self.h, _p(G), G.shape[0],
                                                 mom.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 self._stream()))
        return mom[:self.dim], mom[self.dim:]

    def save(self, path):
        _check(self.L, self.L.airebo_nn_save(self.h, path.encode()))

    # ---- descriptor operators
    def descriptors(self, ctx, x, species, box, periodic=(1, 1, 1)):
        import torch
        x, s, a = self._geo(ctx, x, species, box, periodic)
        G = torch.empty((x.shape[0], self.dim), dtype=torch.float32, device=self.device)
        _check(self.L, self.L.airebo_nn_descriptors(*a, _p(G), self._stream()))
        return G

    def descriptor_jvp(self, ctx, x, species, box, w, periodic=(1, 1, 1)):
        import torch
        x, s, a = self._geo(ctx, x, species, box, periodic)
        w = torch.as_tensor(w, dtype=torch.float32, device=self.device).reshape(-1, 3).contiguous()
        out = torch.empty((x.shape[0], self.dim), dtype=torch.float32, device=self.device)
        _check(self.L, self.L.airebo_nn_descriptor_jvp(*a, _p(w), _p(out), self._stream()))
        return out

    def descriptor_vjp(self, ctx, x, species, box, g, periodic=(1, 1, 1)):
        """F[k] = -g[k] . dG/dx for sets g [k, n, dim]; returns (F [k, n, 3], virial [6])."""
        import torch
        x, s, a = self._geo(ctx, x, species, box, periodic)
        g = torch.as_tensor(g, dtype=torch.float32, device=self.device).reshape(-1, x.shape[0], self.dim)
        g = g.contiguous()
        F = torch.empty((g.shape[0], x.shape[0], 3), dtype=torch.float32, device=self.device)
        w = torch.empty(6, dtype=torch.float64, device=self.device)
        _check(self.L, self.L.airebo_nn_descriptor_vjp(*a, _p(g), g.shape[0], _p(F), _p(w), self._stream()))
        return F, w

    # ---- evaluation, training, dynamics
    def compute(self, ctx, x, species, box, periodic=(1, 1, 1), threshold=0.1, want_spread=False):
        """Returns energy [4] (used, NN mean, far, NN spread), forces [n,3], virial [6] (device),
        the per-atom force spread (device, or None) and info {E_nn, E_far, E_spread, max_spread,
        fallback}."""
        import torch
        x, s, a = self._geo(ctx, x, species, box, periodic)
        n = x.shape[0]
        e = torch.empty(4, dtype=torch.float64, device=self.device)
        f = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty(6, dtype=torch.float64, device=self.device)
        sp = torch.empty(n, dtype=torch.float32, device=self.device) if want_spread else None
        info = (ctypes.c_double * 5)()
        _check(self.L, self.L.airebo_nn_compute(*a, float(threshold), _p(e), _p(f), _p(w),
                                                 _p(sp) if sp is not None else None, info, self._stream()))
        keys = ("E_nn", "E_far", "E_spread", "max_spread", "fallback")
        return e, f, w, sp, dict(zip(keys, list(info)))

    def gradient(self, ctx, x, species, box, f_ref, e_ref, w_force, w_energy, periodic=(1, 1, 1)):
        """Loss per member for one labelled configuration; leaves the gradient on the device."""
        import torch
        x, s, a = self._geo(ctx, x, species, box, periodic)
        f_ref = torch.as_tensor(f_ref, dtype=torch.float64, device=self.device).reshape(-1, 3).contiguous()
        loss = (ctypes.c_double * self.nmodels)()
        _check(self.L, self.L.airebo_nn_gradient(*a, _p(f_ref), float(e_ref), float(w_force), float(w_energy),
                                                  loss, self._stream()))
        return np.array(list(loss))

    def train_step(self, ctx, x, species, box, f_ref, e_ref, w_force, w_energy, lr, periodic=(1, 1, 1)):
        """airebo_nn_train_step: loss per member before one Adam step (beta1 0.9, beta2 0.999, eps 1e-8)."""
        import torch
        x, s, a = self._geo(ctx, x, species, box, periodic)
        f_ref = torch.as_tensor(f_ref, dtype=torch.float64, device=self.device).reshape(-1, 3).contiguous()
        loss = (ctypes.c_double * self.nmodels)()
        _check(self.L, self.L.airebo_nn_train_step(*a, _p(f_ref), float(e_ref), float(w_force), float(w_energy),
                                                    float(lr), loss, self._stream()))
        return np.array(list(loss))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self.L, self.L.airebo_nn_adam(self.h, lr, beta1, beta2, eps, self._stream()))

    def nve(self, ctx, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5, nsteps=10,
            thermo_every=1, threshold=0.1):
        """Velocity Verlet with surrogate forces in place on device tensors x, v.

        Returns (thermo rows, steps evaluated by AIREBO)."""
        import torch
        s = torch.as_tensor(species, dtype=torch.int32, device=self.device).contiguous()
        _state(x, s.shape[0], "x", self.device)
        _state(v, s.shape[0], "v", self.device)
        rows = nsteps // thermo_every + 1 if thermo_every > 0 else 1
        th = torch.zeros((rows, len(THERMO_COLUMNS)), dtype=torch.float64, device=self.device)
        m = (ctypes.c_double * 2)(*masses)
        nfb = ctypes.c_int64()
        _check(self.L, self.L.airebo_nn_nve(self.h, ctx.h, x.shape[0], _p(x), _p(v), _p(s),
                                             _host3(box, ctypes.c_double), _host3(periodic, ctypes.c_int32), m, dt,
                                             nsteps, thermo_every, _p(th), float(threshold), ctypes.byref(nfb),
                                             self._stream()))
        return th, nfb.value

    def profile_nve(self, ctx, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5, nsteps=10,
                    threshold=0.1):
        """Per-kernel device time over nsteps eager surrogate NVE steps: {name: (total ms, launches)}."""
        import torch
        s = torch.as_tensor(species, dtype=torch.int32, device=self.device).contiguous()
        _state(x, s.shape[0], "x", self.device)
        _state(v, s.shape[0], "v", self.device)
        nk = self.L.airebo_kernel_count()
        ms = (ctypes.c_double * nk)()
        cnt = (ctypes.c_int64 * nk)()
        m = (ctypes.c_double * 2)(*masses)
        _check(self.L, self.L.airebo_nn_profile_nve(self.h, ctx.h, x.shape[0], _p(x), _p(v), _p(s),
                                                     _host3(box, ctypes.c_double), _host3(periodic, ctypes.c_int32),
                                                     m, dt, nsteps, float(threshold), ms, cnt, self._stream()))
        return {self.L.airebo_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(nk)}

    def md_begin(self, ctx, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5,
                 threshold=0.1):
        """Start an MD session of `ctx` driven by this surrogate (advance it with ctx.md_run)."""
        import torch
        s = torch.as_tensor(species, dtype=torch.int32, device=self.device).contiguous()
        n = s.shape[0]
        _state(x, n, "x", self.device)
        _state(v, n, "v", self.device)
        m = (ctypes.c_double * 2)(*masses)
        ctx._md = (n, 1, s)
        ctx._md_nn = self   # the surrogate must outlive the session
        _check(self.L, self.L.airebo_nn_md_begin(self.h, ctx.h, n, _p(x), _p(v), _p(s),
                                                 _host3(box, ctypes.c_double), _host3(periodic, ctypes.c_int32), m,
                                                 dt, float(threshold), self._stream()))


def mfma_check(A, B):
    """D = A B for 16x16 FP32 device matrices through the library's matrix-core tile."""
    import torch
    L = load_library()
    D = torch.empty((16, 16), dtype=torch.float32, device=A.device)
    A = A.contiguous()
    B = B.contiguous()
    _check(L, L.airebo_nn_mfma_check(_p(A), _p(B), _p(D),
                                      ctypes.c_void_p(torch.cuda.current_stream(A.device).cuda_stream)))
    return D


def mfma32_check(A, B):
    """D = A B for FP32 device matrices A [16][32], B [32][16] through the
    library's 16x16x32 matrix-core tile."""
    import torch
    L = load_library()
    D = torch.empty((16, 16), dtype=torch.float32, device=A.device)
    A = A.contiguous()
    B = B.contiguous()
    _check(L, L.airebo_nn_mfma32_check(_p(A), _p(B), _p(D),
                                        ctypes.c_void_p(torch.cuda.current_stream(A.device).cuda_stream)))
    return D


def measured_peaks(copy_mib=1024, fma_iters=8192):
    """Measured device peaks: streaming-copy bandwidth (GB/s, bytes read +
    written) and FP64 / FP32 fused multiply-add throughput (TFLOP/s)."""
    import torch
    L = load_library()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = copy_mib * (1 << 20)
    a = torch.empty(n // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    gbs = ctypes.c_double()
    _check(L, L.airebo_peak_copy(_p(a), _p(b), n, 5, ctypes.byref(gbs), st))
    del a, b
    f64, f32 = ctypes.c_double(), ctypes.c_double()
    _check(L, L.airebo_peak_fma(1, fma_iters, ctypes.byref(f64), st))
    _check(L, L.airebo_peak_fma(0, fma_iters, ctypes.byref(f32), st))
    return {"copy_GBps": gbs.value, "fp64_fma_TFLOPs": f64.value, "fp32_fma_TFLOPs": f32.value}
