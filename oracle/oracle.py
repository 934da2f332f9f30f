"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Loads ``oracle/liboracle.so`` (built from ``airebo_oracle.cpp`` by
``oracle.build()`` or ``__graft_entry__.build()``).  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark use this module; the GPU
library never imports it and it never imports the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "airebo_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
DEFAULT_PARAMS = os.path.join(os.path.dirname(HERE), "paper_1810_07026_amd", "params", "airebo_ch.param")

MASK_REBO, MASK_LJ, MASK_TORS, MASK_ALL = 1, 2, 4, 7
MASK_MORSE = 8   # with MASK_LJ: the Morse form of AIREBO-M in place of Lennard-Jones

_lib = None


def build(force=True):
    """Compile the oracle with g++ (OpenMP, -O2)."""
    if force or not os.path.exists(LIB):
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-o", LIB, SRC])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_params_new.restype = ctypes.c_void_p
        L.oracle_params_new.argtypes = [ctypes.c_char_p]
        L.oracle_params_free.argtypes = [ctypes.c_void_p]
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_rc_max.restype = ctypes.c_double
        L.oracle_rc_max.argtypes = [ctypes.c_void_p]
        L.oracle_compute.restype = ctypes.c_int
        L.oracle_compute.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ip, dp, ip, ctypes.c_int, ip,
                                     ctypes.c_int, dp, dp, dp, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.c_int]
        L.oracle_spline.restype = ctypes.c_double
        L.oracle_spline.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
        L.oracle_bond_order.restype = ctypes.c_int
        L.oracle_bond_order.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ip, dp, ip, ctypes.c_int,
                                        ctypes.c_int, dp, ctypes.c_int, dp]
        L.oracle_cij.restype = ctypes.c_double
        L.oracle_cij.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ip, dp, ip, ctypes.c_int,
                                 ctypes.c_int, dp]
        L.oracle_nve.restype = ctypes.c_int
        L.oracle_nve.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, ip, dp, ip, dp, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class OracleError(RuntimeError):
    pass


class Oracle:
    """FP64 AIREBO on the CPU: energies, forces, virial, NVE."""

    def __init__(self, params_path=DEFAULT_PARAMS, nthreads=0):
        self.L = lib()
        self.h = self.L.oracle_params_new(params_path.encode())
        if not self.h:
            raise OracleError(self.L.oracle_last_error().decode())
        self.nthreads = nthreads

    def __del__(self):
        if getattr(self, "h", None):
            self.L.oracle_params_free(self.h)
            self.h = None

    @property
    def rc_max(self):
        return self.L.oracle_rc_max(self.h)

    @staticmethod
    def _prep(x, species, box, periodic):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        s = np.ascontiguousarray(species, dtype=np.int32)
        b = np.ascontiguousarray(box, dtype=np.float64)
        p = np.ascontiguousarray(periodic if periodic is not None else [1, 1, 1], dtype=np.int32)
        return x, s, b, p

    def compute(self, x, species, box, periodic=None, mask=MASK_ALL, sel=None, stats=False):
        """Returns (energy[4] = total, REBO, LJ, torsion; forces[n,3]; virial[6] = xx yy zz xy xz yz)."""
        x, s, b, p = self._prep(x, species, box, periodic)
        n = len(s)
        e = np.zeros(4)
        f = np.zeros((n, 3))
        w = np.zeros(6)
        st = np.zeros(6, dtype=np.int64)
        selp, nsel = None, 0
        if sel is not None:
            sel = np.ascontiguousarray(sel, dtype=np.int32)
            selp, nsel = _i(sel), len(sel)
        rc = self.L.oracle_compute(self.h, n, _d(x), _i(s), _d(b), _i(p), mask, selp, nsel, _d(e), _d(f),
                                   _d(w), st.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                   self.nthreads)
        if rc:
            raise OracleError(self.L.oracle_last_error().decode())
        if stats:
            return e, f, w, dict(zip(["lj_in_cut", "cij_zero", "bstar_needed", "dsb_nonzero", "bonds",
                                      "dihedrals"], st.tolist()))
        return e, f, w

    def energy(self, x, species, box, periodic=None, mask=MASK_ALL):
        return self.compute(x, species, box, periodic, mask)[0][0]

    def spline(self, which, *args):
        a = np.ascontiguousarray(args, dtype=np.float64)
        g = np.zeros(3)
        v = self.L.oracle_spline(self.h, which, _d(a), _d(g))
        return v, g[:len(args)]

    def bond_order(self, x, species, box, i, j, dij=None, bstar=False, periodic=None):
        x, s, b, p = self._prep(x, species, box, periodic)
        if dij is None:
            dij = x[j] - x[i]
        dij = np.ascontiguousarray(dij, dtype=np.float64)
        out = np.zeros(8)
        rc = self.L.oracle_bond_order(self.h, len(s), _d(x), _i(s), _d(b), _i(p), i, j, _d(dij), int(bstar),
                                      _d(out))
        if rc:
            raise OracleError(self.L.oracle_last_error().decode())
        return dict(zip(["b", "pij", "pji", "pirc", "pidh", "Nij", "Nji", "Nconj"], out.tolist()))

    def cij(self, x, species, box, i, j, dij=None, periodic=None):
        x, s, b, p = self._prep(x, species, box, periodic)
        if dij is None:
            dij = x[j] - x[i]
        dij = np.ascontiguousarray(dij, dtype=np.float64)
        return self.L.oracle_cij(self.h, len(s), _d(x), _i(s), _d(b), _i(p), i, j, _d(dij))

    def nve(self, x, v, species, box, masses=(12.011, 1.008), dt=0.5, nsteps=10, thermo_every=1,
            periodic=None):
        """Velocity Verlet; returns (x, v, thermo rows [step, PE, KE, Etot, T, 0])."""
        x, s, b, p = self._prep(x, species, box, periodic)
        x = x.copy()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3).copy()
        m = np.ascontiguousarray(masses, dtype=np.float64)
        nrows = (nsteps // thermo_every + 1) if thermo_every > 0 else 0
        th = np.zeros((max(nrows, 1), 6))
        rc = self.L.oracle_nve(self.h, len(s), _d(x), _d(v), _i(s), _d(b), _i(p), _d(m), dt, nsteps,
                               thermo_every, _d(th), self.nthreads)
        if rc:
            raise OracleError(self.L.oracle_last_error().decode())
        return x, v, th[:nrows]
