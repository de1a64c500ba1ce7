"""Seeded synthetic inputs shared, as data, by the CPU oracle and the GPU library.

Nothing here evaluates the force law or advances time; it produces radii, box
sizes, model parameters and relaxed initial packings with the shapes of the
paper's workloads (Sec. II.E: O(10^3) spheres of radius a and 1.4a in a cubic
periodic box; Table 1 parameters rho = 0.1, eta = 0.1, k_n = 1e4) and of the
larger benchmark configurations.

Parameter readings (the paper does not state them for every configuration):
  * bidisperse = radii 1.0 and 1.4, exactly half of each, ids shuffled;
  * log-normal = ln a ~ N(-0.02, 0.2^2) resampled until inside [0.6, 1.6];
  * box L = (sum 4/3 pi a^3 / phi)^(1/3);
  * Pe = 6 pi eta a^3 gammadot / kT (Sec. II.F) with a = 1; following the
    protocol of Table 1, Pe >= 1 uses gammadot = 0.009 and kT from Pe, Pe < 1
    uses kT = 0.017 and gammadot from Pe; a configuration may fix kT instead;
  * k_t = 2/7 k_n; initial velocities = imposed shear flow + Maxwell-Boltzmann
    at kT, initial spins = -gammadot/2 about z + thermal.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import math
import os
import subprocess
from dataclasses import dataclass, field, asdict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pack.c")
LIB = os.path.join(HERE, "libpack.so")
CACHE = os.environ.get("SUSP_INPUT_CACHE", "/tmp/susp_inputs")

_lib = None
PACK_VERSION = 3   # part of the cache key: packings of an older packer are not reused


def build(force=False):
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _pack():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        _lib.pack_relax.restype = C.c_double
        _lib.pack_relax.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_int, C.c_double, C.POINTER(C.c_int)]
    return _lib


def radii_bidisperse(n, seed):
    rng = np.random.default_rng(seed)
    a = np.where(np.arange(n) < n // 2, 1.0, 1.4)
    rng.shuffle(a)
    return a


def radii_lognormal(n, seed, mu=-0.02, sigma=0.2, lo=0.6, hi=1.6):
    rng = np.random.default_rng(seed)
    out = np.empty(0)
    while out.size < n:
        d = np.exp(rng.normal(mu, sigma, size=int(1.1 * (n - out.size)) + 16))
        out = np.concatenate([out, d[(d >= lo) & (d <= hi)]])
    return out[:n].copy()


def box_length(radii, phi):
    return float((np.sum(4.0 / 3.0 * math.pi * radii ** 3) / phi) ** (1.0 / 3.0))


def pe_to_rates(pe, eta=0.1, kT=None):
    """(gammadot, kT) for a Peclet number Pe = 6 pi eta a^3 gammadot / kT, a = 1."""
    if kT is not None:
        return pe * kT / (6.0 * math.pi * eta), kT
    if pe >= 1.0:
        gd = 0.009
        return gd, 6.0 * math.pi * eta * gd / pe
    kT = 0.017
    return pe * kT / (6.0 * math.pi * eta), kT


def relaxed_positions(radii, L, seed, tol=None, maxiter=20000, alpha=1.2):
    """Uniform random centres, then overlap-removal sweeps until max overlap <= tol."""
    n = len(radii)
    if tol is None:
        tol = 1e-4 * float(np.min(radii))
    key = hashlib.sha1(np.ascontiguousarray(radii).tobytes() + repr((L, seed, tol, alpha, PACK_VERSION)).encode()
                       ).hexdigest()[:20]
    path = os.path.join(CACHE, f"pack_{n}_{key}.npy")
    if os.path.exists(path):
        try:
            return np.load(path)
        except Exception:
            pass
    rng = np.random.default_rng(seed + 7919)
    x = np.ascontiguousarray(rng.random((n, 3)) * L, dtype=np.float64)
    a = np.ascontiguousarray(radii, dtype=np.float64)
    Lb = np.array([L, L, L], dtype=np.float64)
    it = C.c_int(0)
    dp = C.POINTER(C.c_double)
    mo = _pack().pack_relax(n, a.ctypes.data_as(dp), x.ctypes.data_as(dp), Lb.ctypes.data_as(dp),
                            float(tol), int(maxiter), float(alpha), C.byref(it))
    if mo < 0:
        raise RuntimeError(f"packing: more than 64 neighbours of one sphere within the list range")
    if mo > tol:
        raise RuntimeError(f"packing did not relax: max overlap {mo:.3e} > {tol:.3e} after {it.value} sweeps")
    try:
        os.makedirs(CACHE, exist_ok=True)
        np.save(path + ".tmp.npy", x)
        os.replace(path + ".tmp.npy", path)
    except OSError:
        pass
    return x


@dataclass
class Workload:
    name: str
    n: int
    phi: float
    pe: float
    mu: float = 0.5
    radii: str = "bidisperse"        # or "lognormal"
    kT: float | None = None          # fixes kT (then gammadot follows from Pe)
    steps: int = 1000
    seed: int = 0
    rho: float = 0.1
    eta: float = 0.1
    kn: float = 1e4
    dt: float = 1e-4
    xi_cut: float = 0.05
    xi_min: float = 1e-3
    extra: dict = field(default_factory=dict)

    def rates(self):
        return pe_to_rates(self.pe, self.eta, self.kT)

    def params(self):
        gd, kT = self.rates()
        return dict(rho=self.rho, eta=self.eta, kn=self.kn, kt=2.0 * self.kn / 7.0, mu=self.mu, kT=kT,
                    gammadot=gd, dt=self.dt, xi_cut=self.xi_cut, xi_min=self.xi_min, seed=self.seed)


# The five workload shapes used by the tests and the benchmark.
C1 = Workload("bidisperse N=500 phi=0.50 Pe=1 kT=1 FP64", 500, 0.50, 1.0, kT=1.0, steps=1000)
C2 = Workload("bidisperse N=50000 phi=0.55 Pe=10 FP64", 50_000, 0.55, 10.0, steps=10_000)
C3 = Workload("bidisperse N=1000000 phi=0.56 Pe=10 mixed", 1_000_000, 0.56, 10.0, steps=5000)
C5 = Workload("log-normal N=4000000 phi=0.58 Pe=1000 mu=1 mixed", 4_000_000, 0.58, 1000.0, mu=1.0,
              radii="lognormal", steps=10_000)


def sweep_replicas(count=64):
    """Flow-curve sweep: N_r uniform in [2000, 20000] (even), phi cycling over
    {0.45, 0.50, 0.54, 0.58}, Pe log-spaced from 1e-2 to 1e3, seeds 0..count-1."""
    phis = (0.45, 0.50, 0.54, 0.58)
    out = []
    for r in range(count):
        n = 2 * int(np.random.default_rng(1000 + r).integers(1000, 10001))
        pe = 10.0 ** (-2.0 + 5.0 * r / max(count - 1, 1))
        out.append(Workload(f"replica {r}", n, phis[r % 4], pe, seed=r, steps=5000))
    return out


def make_state(w: Workload, n: int | None = None, phi: float | None = None):
    """Radii, box, relaxed positions and thermal initial velocities for a workload."""
    n = w.n if n is None else n
    phi = w.phi if phi is None else phi
    if w.radii == "lognormal":
        a = radii_lognormal(n, w.seed)
    else:
        a = radii_bidisperse(n, w.seed)
    L = box_length(a, phi)
    x = relaxed_positions(a, L, w.seed)
    gd, kT = w.rates()
    rng = np.random.default_rng(w.seed + 104729)
    m = 4.0 / 3.0 * math.pi * w.rho * a ** 3
    inertia = 0.4 * m * a ** 2
    v = rng.standard_normal((n, 3)) * np.sqrt(kT / m)[:, None]
    v[:, 0] += gd * (x[:, 1] - 0.5 * L)
    om = rng.standard_normal((n, 3)) * np.sqrt(kT / inertia)[:, None]
    om[:, 2] += -0.5 * gd
    return dict(radii=a, x=x, v=v, w=om, L=(L, L, L), params=w.params(), n=n, phi=phi)


def random_state(n, L, radii, seed, kT=1.0, gammadot=0.0, rho=0.1):
    """Unrelaxed uniform random centres (overlaps allowed) for small geometric tests."""
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)) * np.asarray(L)[None, :]
    m = 4.0 / 3.0 * math.pi * rho * radii ** 3
    v = rng.standard_normal((n, 3)) * np.sqrt(kT / m)[:, None]
    v[:, 0] += gammadot * (x[:, 1] - 0.5 * L[1])
    w = rng.standard_normal((n, 3)) * np.sqrt(kT / (0.4 * m * radii ** 2))[:, None]
    return x, v, w
