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

FP64, MIXED = 0, 1
TERM_REBO, TERM_LJ, TERM_TORSION, TERM_ALL = 1, 2, 4, 7
STAT_NAMES = ["lj_in_cut", "cij_zero", "bstar_queued", "dsb_nonzero", "bonds", "rebuilds", "max_short",
              "reserved7", "max_lj", "spline_evals", "spline_evals_fp64"]

EXPORTS = ["airebo_options_default", "airebo_ctx_create", "airebo_ctx_free", "airebo_compute", "airebo_nve",
           "airebo_stats", "airebo_last_error", "airebo_profile_nve", "airebo_kernel_count", "airebo_kernel_name",
           "airebo_batch_compute", "airebo_batch_nve"]


class AireboError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"airebo error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("term_mask", ctypes.c_int32), ("skin", ctypes.c_double),
                ("lj_cap", ctypes.c_int32), ("device", ctypes.c_int32), ("bond_block", ctypes.c_int32),
                ("bond_grid", ctypes.c_int32), ("defer_block", ctypes.c_int32), ("short_block", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]

    TUNABLES = ("bond_block", "bond_grid", "defer_block", "short_block")


_lib = None


def load_library(path=LIB_PATH):
    """Load libairebo.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise AireboError(-1, f"{path} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
    L.airebo_options_default.argtypes = [ctypes.POINTER(Options)]
    L.airebo_options_default.restype = None
    L.airebo_ctx_create.argtypes = [ctypes.c_char_p, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]
    L.airebo_ctx_create.restype = ctypes.c_int
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
    L.airebo_last_error.argtypes = []
    L.airebo_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(L, rc):
    if rc != 0:
        raise AireboError(rc, L.airebo_last_error().decode())


def _host3(a, ctype):
    arr = (ctype * 3)(*a)
    return arr


class Context:
    """One AIREBO evaluation context on one GPU."""

    def __init__(self, params=DEFAULT_PARAMS, precision=FP64, term_mask=TERM_ALL, skin=1.0, lj_cap=0, device=0,
                 tune=None):
        import torch
        if not torch.cuda.is_available():
            raise AireboError(-7, "no GPU visible: the AIREBO library runs on the GPU only")
        self.L = load_library()
        o = Options()
        self.L.airebo_options_default(ctypes.byref(o))
        o.precision, o.term_mask, o.skin, o.lj_cap, o.device = precision, term_mask, skin, lj_cap, device
        for k, v in (tune or {}).items():
            if k not in Options.TUNABLES:
                raise AireboError(-1, f"unknown tunable {k}")
            setattr(o, k, int(v))
        self.tune = dict(tune or {})
        h = ctypes.c_void_p()
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

    def nve(self, x, v, species, box, periodic=(1, 1, 1), masses=(12.011, 1.008), dt=0.5, nsteps=10,
            thermo_every=1):
        """Velocity Verlet in place on device tensors x, v; returns the thermo rows (device tensor)."""
        import torch
        assert x.is_cuda and v.is_cuda and x.dtype == torch.float64 and v.dtype == torch.float64
        s = self._dev(species, torch.int32)
        n = x.shape[0]
        rows = nsteps // thermo_every + 1 if thermo_every > 0 else 1
        th = torch.zeros((rows, 6), dtype=torch.float64, device=self.device)
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
        assert x.is_cuda and v.is_cuda
        s = self._dev(species, torch.int32)
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
        """Batched velocity Verlet in place; returns thermo [rows, nsys, 6] (device tensor)."""
        import torch
        assert x.is_cuda and v.is_cuda
        s = self._dev(species, torch.int32)
        nsys, off, b, p = self._batch_host(sizes, boxes, periodic)
        rows = nsteps // thermo_every + 1 if thermo_every > 0 else 1
        th = torch.zeros((rows, nsys, 6), dtype=torch.float64, device=self.device)
        m = (ctypes.c_double * 2)(*masses)
        rc = self.L.airebo_batch_nve(
            self.h, nsys, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(s.data_ptr()), m, dt,
            nsteps, thermo_every, ctypes.c_void_p(th.data_ptr()), self._stream())
        _check(self.L, rc)
        return th

    def stats(self):
        out = (ctypes.c_int64 * 16)()
        _check(self.L, self.L.airebo_stats(self.h, out))
        return dict(zip(STAT_NAMES, list(out)[:len(STAT_NAMES)]))
