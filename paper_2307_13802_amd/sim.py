"""ctypes binding of ``include/sim.h``: same names, argument marshalling only.

Every step of the physics runs inside ``libsusp.so`` on the GPU; if the
library has not been built, loading fails with an error instead of falling
back to anything else.  PyTorch, when present, supplies the HIP stream and
(optionally) the caching allocator.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "sim.h")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ECAPACITY, ERANGE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
FREEZE_X, NO_LUB, NO_PAIR_BROWN, NO_CONTACT, NO_ONEBODY, LUB_ROT = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
REBUILD_EACH_STEP, NO_GRAPH = 0x100, 0x200
HALF_OCC_ON, HALF_OCC_OFF = 0x400, 0x800  # half-pair kernel, FP64: force or forbid its form for occupancy
SMALL_QUEUE = 0x1000  # test switch: that form's pair queue in rounds of 64 items
TRACK_DISPLACEMENT = 0x2000  # keep each particle's non-affine displacement (sim_displacement, sim_msd)
KERNEL_AUTO, KERNEL_HALF = 0, 3
STRESS_CONTACT, STRESS_LUB, STRESS_BROWN, STRESS_DRAG, STRESS_TOTAL = range(5)
STRESS_LAST, STRESS_MEAN = 0, 1


def library_path() -> str:
    return os.path.join(HERE, "libsusp.so")


def build(verbose=False) -> str:
    from . import build_lib as _b
    return _b.build(verbose=verbose)


class _Config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n", C.c_uint32), ("box", C.c_double * 3), ("rho", C.c_double),
                ("eta", C.c_double), ("kn", C.c_double), ("kt", C.c_double), ("mu", C.c_double),
                ("kT", C.c_double), ("gammadot", C.c_double), ("dt", C.c_double), ("xi_cut", C.c_double),
                ("xi_min", C.c_double), ("skin", C.c_double), ("le_offset0", C.c_double),
                ("max_overlap", C.c_double), ("repulsion", C.c_double), ("cell_factor", C.c_double),
                ("seed", C.c_uint64), ("step0", C.c_uint64),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("nlist_cap", C.c_uint32),
                ("lanes", C.c_uint32), ("pair_kernel", C.c_uint32), ("reserved", C.c_uint32)]


class _Stats(C.Structure):
    _fields_ = [("contacts_per_particle", C.c_double), ("sliding_fraction", C.c_double),
                ("max_overlap", C.c_double), ("neighbours_per_particle", C.c_double),
                ("interacting_per_particle", C.c_double), ("contacts", C.c_int64), ("rebuilds", C.c_int64),
                ("steps", C.c_int64), ("step", C.c_uint64), ("le_offset", C.c_double), ("lanes", C.c_int32),
                ("pair_kernel", C.c_int32), ("occupancy_form", C.c_int32), ("tune_source", C.c_int32),
                ("skin", C.c_double), ("cell_factor", C.c_double), ("kT_translational", C.c_double),
                ("kT_rotational", C.c_double), ("cells_x", C.c_int32), ("cells_y", C.c_int32),
                ("cells_z", C.c_int32), ("list_cap", C.c_int32)]


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None
_ALLOC_CB = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_CB = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_keep = []


def lib():
    """Loads libsusp.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2307_13802_amd.build() (hipcc, gfx950)")
    L = C.CDLL(path)
    dp, up, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    vp = C.c_void_p
    sig = {
        "sim_validate": [C.POINTER(_Config), dp],
        "sim_create": [C.POINTER(_Config), C.c_int32, C.POINTER(dp), C.POINTER(dp), C.POINTER(dp), C.POINTER(dp),
                       vp, C.POINTER(vp)],
        "sim_step": [vp, C.c_int64],
        "sim_stress": [vp, C.c_int32, C.c_int32, C.c_int32, dp],
        "sim_reset_stress": [vp],
        "sim_stress_series": [vp, C.c_int32, dp, C.c_int64, lp],
        "sim_positions": [vp, C.c_int32, dp],
        "sim_structural_stress": [vp, C.c_int32, dp],
        "sim_displacement": [vp, C.c_int32, dp],
        "sim_msd": [vp, C.c_int32, dp],
        "sim_reset_displacement": [vp],
        "sim_rdf": [vp, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_uint64)],
        "sim_rdf_xy": [vp, C.c_int32, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_uint64)],
        "sim_rdf_noalloc": [vp, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_uint64)],
        "sim_stress_acf_stream": [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int64],
        "sim_stress_acf": [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64, dp],
        "sim_get_state": [vp, C.c_int32, dp, dp, dp, dp, dp, dp, C.POINTER(C.c_uint64)],
        "sim_set_state": [vp, C.c_int32, dp, dp, dp, dp, dp, C.c_double, C.c_uint64, up, dp, C.c_int64],
        "sim_forces": [vp, C.c_int32, dp, dp],
        "sim_pairs": [vp, C.c_int32, up, C.c_int64, lp],
        "sim_nlist": [vp, C.c_int32, up, C.c_int64, lp],
        "sim_contacts": [vp, C.c_int32, up, dp, ip, C.c_int64, lp],
        "sim_stats": [vp, C.c_int32, C.POINTER(_Stats)],
        "sim_profile": [vp, C.c_int32],
        "sim_kernel_time": [vp, lp, dp],
        "sim_stage_time": [vp, C.c_int32, lp, dp],
        "sim_destroy": [vp],
        "sim_last_error": [vp, C.c_char_p, C.c_size_t],
        "sim_set_allocator": [_ALLOC_CB, _FREE_CB, vp],
        "sim_set_tune_cache": [C.c_char_p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.sim_strerror.argtypes = [C.c_int32]
    L.sim_strerror.restype = C.c_char_p
    _lib = L
    return L


def _err(handle=None):
    buf = C.create_string_buffer(1024)
    lib().sim_last_error(handle, buf, 1024)
    return buf.value.decode(errors="replace")


def _check(rc, handle=None):
    if rc != OK:
        raise SimError(rc, f"{lib().sim_strerror(rc).decode()}: {_err(handle)}")


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


@dataclass
class Config:
    """Mirror of ``sim_config``: model inputs of Sec. II.E/II.F plus numerics."""
    box: tuple
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
    skin: float = 0.0
    le_offset0: float = 0.0
    max_overlap: float = 0.0
    repulsion: float = 0.0
    cell_factor: float = 0.0
    seed: int = 0
    step0: int = 0
    precision: int = FP64
    flags: int = 0
    nlist_cap: int = 0
    lanes: int = 0
    pair_kernel: int = 0

    def c(self, n) -> _Config:
        c = _Config()
        c.struct_size = C.sizeof(_Config)
        c.n = int(n)
        for d in range(3):
            c.box[d] = float(self.box[d])
        for f in ("rho", "eta", "kn", "kt", "mu", "kT", "gammadot", "dt", "xi_cut", "xi_min", "skin",
                  "le_offset0", "max_overlap", "repulsion", "cell_factor"):
            setattr(c, f, float(getattr(self, f)))
        c.seed, c.step0 = int(self.seed), int(self.step0)
        c.precision, c.flags, c.nlist_cap = int(self.precision), int(self.flags), int(self.nlist_cap)
        c.lanes = int(self.lanes)
        c.pair_kernel = int(self.pair_kernel)
        c.reserved = 0
        return c


def validate(cfg: Config, radii) -> int:
    a = np.ascontiguousarray(radii, dtype=np.float64)
    c = cfg.c(len(a))
    return lib().sim_validate(C.byref(c), _dp(a))


def set_tune_cache(path):
    """Cache file of tuned launch and list parameters for later handles (None = none)."""
    _check(lib().sim_set_tune_cache(None if path is None else str(path).encode()))


def last_error() -> str:
    return _err(None)


def use_torch_allocator():
    """Routes device allocations of later handles through torch's caching allocator."""
    import torch

    def _alloc(nbytes, ctx):
        return int(torch.cuda.caching_allocator_alloc(int(nbytes)))

    def _free(p, ctx):
        torch.cuda.caching_allocator_delete(p)

    a, f = _ALLOC_CB(_alloc), _FREE_CB(_free)
    _keep.extend([a, f])
    _check(lib().sim_set_allocator(a, f, None))


def use_default_allocator():
    """Routes device allocations of later handles to hipMalloc / hipFree again."""
    _check(lib().sim_set_allocator(_ALLOC_CB(), _FREE_CB(), None))


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(None)


class Sim:
    """One handle: R replicas advanced together on one GPU."""

    def __init__(self, configs, radii, x0, v0=None, w0=None, stream=None):
        if isinstance(configs, Config):
            configs, radii, x0 = [configs], [radii], [x0]
            v0 = None if v0 is None else [v0]
            w0 = None if w0 is None else [w0]
        R = len(configs)
        self.n = [int(len(a)) for a in radii]
        self._keep = []
        arr = (_Config * R)(*[cfg.c(n) for cfg, n in zip(configs, self.n)])
        self.configs = list(configs)

        def ptrs(seq):
            if seq is None:
                return None
            out = (C.POINTER(C.c_double) * R)()
            for r, a in enumerate(seq):
                if a is None:
                    out[r] = C.POINTER(C.c_double)()
                    continue
                a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                self._keep.append(a)
                out[r] = _dp(a)
            return out

        self.radii = [np.ascontiguousarray(a, dtype=np.float64) for a in radii]
        h = C.c_void_p()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        rc = lib().sim_create(arr, R, ptrs(self.radii), ptrs(x0), ptrs(v0), ptrs(w0), st, C.byref(h))
        self._keep = []
        _check(rc)
        self.h = h

    # -- lifetime
    def close(self):
        if getattr(self, "h", None):
            lib().sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- stepping and observables
    def step(self, nsteps=1):
        _check(lib().sim_step(self.h, int(nsteps)), self.h)

    def stress(self, replica=0, component=STRESS_TOTAL, mode=STRESS_LAST):
        out = np.zeros(9)
        _check(lib().sim_stress(self.h, replica, component, mode, _dp(out)), self.h)
        return out.reshape(3, 3)

    def reset_stress(self):
        _check(lib().sim_reset_stress(self.h), self.h)

    def stress_series(self, replica=0):
        cnt = C.c_int64(0)
        rc = lib().sim_stress_series(self.h, replica, None, 0, C.byref(cnt))
        if rc not in (OK, ERANGE):
            _check(rc, self.h)
        out = np.zeros((max(cnt.value, 1), 27))
        _check(lib().sim_stress_series(self.h, replica, _dp(out), cnt.value, C.byref(cnt)), self.h)
        return out[: cnt.value].reshape(-1, 3, 3, 3)

    def structural_stress(self, replica=0):
        """Structural Brownian stress of the current configuration (3x3)."""
        out = np.zeros(9)
        _check(lib().sim_structural_stress(self.h, replica, _dp(out)), self.h)
        return out.reshape(3, 3)

    def displacement(self, replica=0):
        """Accumulated non-affine displacement per particle, (n, 3), id order."""
        out = np.zeros((self.n[replica], 3))
        _check(lib().sim_displacement(self.h, replica, _dp(out)), self.h)
        return out

    def msd(self, replica=0):
        """Mean square of the accumulated displacement per axis, (3,)."""
        out = np.zeros(3)
        _check(lib().sim_msd(self.h, replica, _dp(out)), self.h)
        return out

    def reset_displacement(self):
        _check(lib().sim_reset_displacement(self.h), self.h)

    def rdf(self, r_max, nbins, replica=0):
        """Pair-distance histogram of the current configuration (counts per bin)."""
        out = np.zeros(nbins, np.uint64)
        _check(lib().sim_rdf(self.h, replica, float(r_max), int(nbins), out.ctypes.data_as(C.POINTER(C.c_uint64))),
               self.h)
        return out

    def rdf_noalloc(self, r_max, nbins, replica=0):
        """sim_rdf with its bins in the library's static device array (no device allocation)."""
        out = np.zeros(nbins, np.uint64)
        _check(lib().sim_rdf_noalloc(self.h, replica, float(r_max), int(nbins),
                                     out.ctypes.data_as(C.POINTER(C.c_uint64))), self.h)
        return out

    def rdf_xy(self, r_max, slab, nbins, replica=0):
        """Pair counts in the flow-gradient slice |r_z| < slab/2, (nbins, nbins) over [-r_max, r_max)^2."""
        out = np.zeros(nbins * nbins, np.uint64)
        _check(lib().sim_rdf_xy(self.h, replica, float(r_max), float(slab), int(nbins),
                                out.ctypes.data_as(C.POINTER(C.c_uint64))), self.h)
        return out.reshape(nbins, nbins)

    def stress_acf_stream(self, component, alpha, beta, nlag):
        """Accumulates the autocorrelation of a stress entry on the device at every recorded step."""
        _check(lib().sim_stress_acf_stream(self.h, component, alpha, beta, int(nlag)), self.h)

    def stress_acf(self, component, alpha, beta, nlag, replica=0):
        """Time autocorrelation of a recorded stress entry over the records since the reset."""
        out = np.zeros(nlag)
        _check(lib().sim_stress_acf(self.h, replica, component, alpha, beta, int(nlag), _dp(out)), self.h)
        return out

    def positions(self, replica=0):
        out = np.zeros((self.n[replica], 3))
        _check(lib().sim_positions(self.h, replica, _dp(out)), self.h)
        return out

    def get_state(self, replica=0):
        n = self.n[replica]
        x, v, w, F, T = (np.zeros((n, 3)) for _ in range(5))
        s = C.c_double(0)
        k = C.c_uint64(0)
        _check(lib().sim_get_state(self.h, replica, _dp(x), _dp(v), _dp(w), _dp(F), _dp(T), C.byref(s),
                                   C.byref(k)), self.h)
        return dict(x=x, v=v, w=w, F=F, T=T, s_le=s.value, step=k.value)

    def set_state(self, replica, x, v, w, F=None, T=None, s_le=0.0, step=0, contacts=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        Fp = Tp = None
        if F is not None:
            F = np.ascontiguousarray(F, dtype=np.float64)
            T = np.ascontiguousarray(T, dtype=np.float64)
            Fp, Tp = _dp(F), _dp(T)
        if contacts is not None and len(contacts[0]):
            cij = np.ascontiguousarray(contacts[0], dtype=np.uint32)
            cs = np.ascontiguousarray(contacts[1], dtype=np.float64)
            nc = len(cij)
            cp, sp = _up(cij), _dp(cs)
        else:
            nc, cp, sp = 0, None, None
        _check(lib().sim_set_state(self.h, replica, _dp(x), _dp(v), _dp(w), Fp, Tp, float(s_le), int(step),
                                   cp, sp, nc), self.h)

    def forces(self, replica=0):
        n = self.n[replica]
        F, T = np.zeros((n, 3)), np.zeros((n, 3))
        _check(lib().sim_forces(self.h, replica, _dp(F), _dp(T)), self.h)
        return F, T

    def _pairs(self, fn, replica):
        cnt = C.c_int64(0)
        rc = fn(self.h, replica, None, 0, C.byref(cnt))
        if rc not in (OK, ERANGE):
            _check(rc, self.h)
        out = np.zeros((max(cnt.value, 1), 2), np.uint32)
        _check(fn(self.h, replica, _up(out), cnt.value, C.byref(cnt)), self.h)
        return out[: cnt.value]

    def pairs(self, replica=0):
        return self._pairs(lib().sim_pairs, replica)

    def nlist(self, replica=0):
        return self._pairs(lib().sim_nlist, replica)

    def contacts(self, replica=0):
        cnt = C.c_int64(0)
        rc = lib().sim_contacts(self.h, replica, None, None, None, 0, C.byref(cnt))
        if rc not in (OK, ERANGE):
            _check(rc, self.h)
        m = max(cnt.value, 1)
        ij, s, sl = np.zeros((m, 2), np.uint32), np.zeros((m, 3)), np.zeros(m, np.int32)
        _check(lib().sim_contacts(self.h, replica, _up(ij), _dp(s), sl.ctypes.data_as(C.POINTER(C.c_int32)),
                                  cnt.value, C.byref(cnt)), self.h)
        k = cnt.value
        return ij[:k], s[:k], sl[:k]

    def stats(self, replica=0):
        st = _Stats()
        _check(lib().sim_stats(self.h, replica, C.byref(st)), self.h)
        return {f: getattr(st, f) for f, _ in _Stats._fields_}

    def profile(self, enable=True):
        _check(lib().sim_profile(self.h, 1 if enable else 0), self.h)

    def kernel_time(self):
        n, ms = C.c_int64(0), C.c_double(0)
        _check(lib().sim_kernel_time(self.h, C.byref(n), C.byref(ms)), self.h)
        return n.value, ms.value

    def stage_time(self, stage):
        """(steps timed, total ms) of one stage: 0 integrate, 1 pair kernel, 2 gather."""
        n, ms = C.c_int64(0), C.c_double(0)
        _check(lib().sim_stage_time(self.h, int(stage), C.byref(n), C.byref(ms)), self.h)
        return n.value, ms.value


def header_functions():
    """Names of the functions declared in include/sim.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(sim_\w+)\s*\(", txt, flags=re.M)))
