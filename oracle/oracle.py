"""ctypes front end of the FP64 CPU oracle (``orc.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module to obtain expected values.  The GPU
library never imports it and shares no code with it.

The oracle follows the paper section by section (Li, Royer & Ness, arXiv
2307.13802): the force law of Sec. II.A-II.D, velocity-Verlet of Sec. II and
the sheared periodic box of Sec. II.E.  See ``orc.c`` for the readings taken
where the text is silent or garbled.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")

FREEZE_X = 0x1
NO_LUB = 0x2
NO_PAIR_BROWN = 0x4
NO_CONTACT = 0x8
NO_ONEBODY = 0x10
CELLS = 0x20
LUB_ROT = 0x40


def build(force: bool = False) -> str:
    """Compile the oracle with IEEE FP64 semantics (no contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("rho", C.c_double), ("eta", C.c_double), ("kn", C.c_double),
                ("kt", C.c_double), ("mu", C.c_double), ("kT", C.c_double), ("gammadot", C.c_double),
                ("dt", C.c_double), ("xi_cut", C.c_double), ("xi_min", C.c_double), ("rep_A", C.c_double),
                ("seed", C.c_uint64), ("flags", C.c_uint32), ("pad", C.c_uint32)]


_lib = None
_lib_lock = threading.Lock()


def lib():
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:
        if _lib is None:
            _lib = _load()
    return _lib


def _load():
    """Loads the compiled oracle and declares its C signatures."""
    _lib = C.CDLL(build())
    dp = C.POINTER(C.c_double)
    up = C.POINTER(C.c_uint32)
    _lib.orc_new.restype = C.c_void_p
    _lib.orc_new.argtypes = [C.POINTER(_Params), C.c_int, dp, dp, dp, dp, C.c_double, C.c_uint64,
                             C.c_int, up, dp, dp, dp]
    _lib.orc_free.argtypes = [C.c_void_p]
    _lib.orc_step.argtypes = [C.c_void_p, C.c_long, dp]
    _lib.orc_eval.argtypes = [C.c_void_p]
    _lib.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp, C.POINTER(C.c_uint64)]
    _lib.orc_get_norms.argtypes = [C.c_void_p, dp, dp]
    _lib.orc_get_stress.argtypes = [C.c_void_p, dp]
    _lib.orc_get_stress_all.argtypes = [C.c_void_p, dp]
    _lib.orc_eta_r.restype = C.c_double
    _lib.orc_eta_r.argtypes = [C.c_void_p]
    _lib.orc_acf.argtypes = [dp, C.c_long, C.c_long, dp]
    _lib.orc_run_rdf.argtypes = [C.c_void_p, C.c_long, C.c_long, C.c_double, C.c_int, C.POINTER(C.c_uint64)]
    _lib.orc_structural_stress.argtypes = [C.c_void_p, dp]
    _lib.orc_get_disp.argtypes = [C.c_void_p, dp]
    _lib.orc_rdf.argtypes = [C.c_void_p, C.c_double, C.c_int, C.POINTER(C.c_uint64)]
    _lib.orc_rdf_xy.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_uint64)]
    _lib.orc_lub_rot_scalars.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
    _lib.orc_get_contacts.restype = C.c_int
    _lib.orc_get_contacts.argtypes = [C.c_void_p, C.c_int, up, dp, C.POINTER(C.c_int32)]
    _lib.orc_get_pairs.restype = C.c_int
    _lib.orc_get_pairs.argtypes = [C.c_void_p, C.c_int, up]
    _lib.orc_verlet_pairs.restype = C.c_long
    _lib.orc_verlet_pairs.argtypes = [C.c_void_p, C.c_double, C.c_long, up]
    _lib.orc_particle_force.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp]
    _lib.orc_philox4x32_10.argtypes = [up, up, up]
    _lib.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, dp]
    _lib.orc_lub_scalars.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


@dataclass
class Params:
    """Model inputs of Sec. II.E/II.F (a, L, rho, k_n, kT, eta, gammadot) plus mu, dt and the gap cut-offs."""
    L: tuple
    rho: float = 0.1
    eta: float = 0.1
    kn: float = 1e4
    kt: float = 2.0 * 1e4 / 7.0
    mu: float = 0.5
    kT: float = 1.0
    gammadot: float = 0.0
    dt: float = 1e-4
    xi_cut: float = 0.05
    xi_min: float = 1e-3
    rep_A: float = 0.0
    seed: int = 0
    flags: int = 0

    def c(self) -> _Params:
        p = _Params()
        for d in range(3):
            p.L[d] = float(self.L[d])
        for f in ("rho", "eta", "kn", "kt", "mu", "kT", "gammadot", "dt", "xi_cut", "xi_min", "rep_A"):
            setattr(p, f, float(getattr(self, f)))
        p.seed = int(self.seed)
        p.flags = int(self.flags)
        return p


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_u(c), _u(k), _u(out))
    return out


def gauss3(seed, c0, c1, c2, c3):
    g = np.zeros(3)
    lib().orc_gauss3(seed, c0, c1, c2, c3, _d(g))
    return g


def lub_scalars(eta, ai, aj, xi):
    xa = np.zeros(1)
    ya = np.zeros(1)
    lib().orc_lub_scalars(eta, ai, aj, xi, _d(xa), _d(ya))
    return float(xa[0]), float(ya[0])


def acf(series, nlag):
    """Time autocorrelation out[k] = mean_t s(t) s(t + k), k < nlag (Sec. IV.B)."""
    s = np.ascontiguousarray(series, dtype=np.float64).reshape(-1)
    out = np.zeros(int(nlag))
    lib().orc_acf(_d(s), len(s), int(nlag), _d(out))
    return out


def lub_rot_scalars(eta, ai, aj, xi):
    """(Y^B_11, Y^B_21, Y^C_11, Y^C_12, Y^C_21, Y^C_22) of Sec. II.B."""
    out = np.zeros(6)
    lib().orc_lub_rot_scalars(eta, ai, aj, xi, _d(out))
    return tuple(float(t) for t in out)


class Oracle:
    """One system.  Particle ids are the array indices 0..n-1."""

    def __init__(self, params: Params, radii, x, v, w, s_le=0.0, step=0, contacts=None, F=None, T=None):
        self.params = params
        self._p = params.c()
        self.n = int(len(radii))
        self.a = np.ascontiguousarray(radii, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        if contacts is None:
            cij = np.zeros(2, np.uint32)
            cs = np.zeros(3)
            nc = 0
        else:
            cij = np.ascontiguousarray(contacts[0], dtype=np.uint32).reshape(-1)
            cs = np.ascontiguousarray(contacts[1], dtype=np.float64).reshape(-1)
            nc = len(cij) // 2
            if nc == 0:
                cij = np.zeros(2, np.uint32)
                cs = np.zeros(3)
        Fp = Tp = None
        if F is not None:
            Fa = np.ascontiguousarray(F, dtype=np.float64).reshape(-1)
            Ta = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
            Fp, Tp = _d(Fa), _d(Ta)
        self._h = lib().orc_new(C.byref(self._p), self.n, _d(self.a), _d(x), _d(v), _d(w), float(s_le),
                                int(step), nc, _u(cij), _d(cs), Fp, Tp)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def step(self, nsteps=1, series=False):
        out = np.zeros((nsteps, 27)) if series else None
        lib().orc_step(self._h, int(nsteps), _d(out) if series else None)
        return out

    def eval(self):
        lib().orc_eval(self._h)

    def state(self):
        n = self.n
        x, v, w, F, T = (np.zeros((n, 3)) for _ in range(5))
        s = np.zeros(1)
        k = C.c_uint64(0)
        lib().orc_get_state(self._h, _d(x), _d(v), _d(w), _d(F), _d(T), _d(s), C.byref(k))
        return dict(x=x, v=v, w=w, F=F, T=T, s_le=float(s[0]), step=int(k.value))

    def norms(self):
        Fa = np.zeros(self.n)
        Ta = np.zeros(self.n)
        lib().orc_get_norms(self._h, _d(Fa), _d(Ta))
        return Fa, Ta

    def stress(self):
        """(3, 3, 3): [contact, lubrication, Brownian] x alpha x beta, Sec. II.A/II.B/II.D."""
        out = np.zeros(27)
        lib().orc_get_stress(self._h, _d(out))
        return out.reshape(3, 3, 3)

    def stress_all(self):
        """(5, 3, 3): contact, lubrication, Brownian, drag stresslet and total (hydrodynamic +
        contact), Sec. II.A-II.D, IV.D."""
        out = np.zeros(45)
        lib().orc_get_stress_all(self._h, _d(out))
        return out.reshape(5, 3, 3)

    def eta_r(self):
        """Relative viscosity of the last evaluation, Sec. II.E."""
        return float(lib().orc_eta_r(self._h))

    def run_rdf(self, nsteps, every, r_max, nbins, counts=None):
        """Runs nsteps steps, adding the pair-distance histogram after every `every`-th step."""
        out = np.zeros(nbins, np.uint64) if counts is None else counts
        lib().orc_run_rdf(self._h, int(nsteps), int(every), float(r_max), int(nbins),
                          out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    def displacement(self):
        """(n, 3) accumulated non-affine displacement (drift minus the imposed flow)."""
        out = np.zeros((self.n, 3))
        lib().orc_get_disp(self._h, _d(out))
        return out

    def rdf(self, r_max, nbins):
        """Pair-distance histogram (each pair once, r < r_max)."""
        out = np.zeros(nbins, np.uint64)
        lib().orc_rdf(self._h, float(r_max), int(nbins), out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out

    def rdf_xy(self, r_max, slab, nbins):
        """Pair counts in the flow-gradient slice |r_z| < slab/2, (nbins, nbins) over [-r_max, r_max)^2."""
        out = np.zeros(nbins * nbins, np.uint64)
        lib().orc_rdf_xy(self._h, float(r_max), float(slab), int(nbins), out.ctypes.data_as(C.POINTER(C.c_uint64)))
        return out.reshape(nbins, nbins)

    def structural_stress(self):
        """(3, 3) structural Brownian stress of the current configuration, Sec. II.D."""
        out = np.zeros(9)
        lib().orc_structural_stress(self._h, _d(out))
        return out.reshape(3, 3)

    def contacts(self):
        n = lib().orc_get_contacts(self._h, 0, _u(np.zeros(2, np.uint32)), _d(np.zeros(3)), None)
        ij = np.zeros((max(n, 1), 2), np.uint32)
        s = np.zeros((max(n, 1), 3))
        sl = np.zeros(max(n, 1), np.int32)
        lib().orc_get_contacts(self._h, n, _u(ij), _d(s), sl.ctypes.data_as(C.POINTER(C.c_int32)))
        return ij[:n], s[:n], sl[:n]

    def pairs(self):
        n = lib().orc_get_pairs(self._h, 0, _u(np.zeros(2, np.uint32)))
        ij = np.zeros((max(n, 1), 2), np.uint32)
        lib().orc_get_pairs(self._h, n, _u(ij))
        return ij[:n]

    def verlet_pairs(self, skin):
        n = lib().orc_verlet_pairs(self._h, float(skin), 0, _u(np.zeros(2, np.uint32)))
        ij = np.zeros((max(n, 1), 2), np.uint32)
        lib().orc_verlet_pairs(self._h, float(skin), n, _u(ij))
        return ij[:n]

    def particle_force(self, i):
        F = np.zeros(3)
        T = np.zeros(3)
        fa = np.zeros(1)
        ta = np.zeros(1)
        lib().orc_particle_force(self._h, int(i), _d(F), _d(T), _d(fa), _d(ta))
        return F, T, float(fa[0]), float(ta[0])
