"""Host-side checks of the C ABI: the library loads without a GPU, exports every
function include/sim.h declares, and validates configurations on the host."""
import ctypes as C
import subprocess

import numpy as np
import pytest

import paper_2307_13802_amd as P
from paper_2307_13802_amd import sim as S


def test_library_exports_every_declared_symbol():
    names = S.header_functions()
    assert len(names) >= 20
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", P.library_path()]).decode()
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_struct_size_matches_header():
    # compile a tiny host program against the public header and compare layouts
    import os
    import tempfile
    d = tempfile.mkdtemp()
    src = os.path.join(d, "t.c")
    open(src, "w").write('#include "sim.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(){printf("%zu %zu %zu %zu\\n",'
                         ' sizeof(sim_config), offsetof(sim_config, seed), offsetof(sim_config, flags),'
                         ' sizeof(sim_stats_t)); return 0;}\n')
    exe = os.path.join(d, "t")
    subprocess.check_call(["gcc", "-I", os.path.join(S.ROOT, "include"), src, "-o", exe])
    size, off_seed, off_flags, ssize = (int(t) for t in subprocess.check_output([exe]).split())
    assert size == C.sizeof(S._Config)
    assert off_seed == S._Config.seed.offset and off_flags == S._Config.flags.offset
    assert ssize == C.sizeof(S._Stats)


def _cfg(**kw):
    c = P.Config(box=(20.0, 20.0, 20.0))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_validate_accepts_good_config():
    a = np.full(10, 1.0)
    assert S.validate(_cfg(), a) == S.OK
    # list range 2 * 1.025 + 0.2 = 2.25 (< 5 / 2), or 2.05 + 0.1 with the smallest tuned skin
    assert S.validate(_cfg(box=(5.0, 20.0, 20.0)), a) == S.OK
    assert S.validate(_cfg(box=(4.4, 20.0, 20.0), skin=-1.0), a) == S.OK
    assert S.validate(_cfg(cell_factor=-1.0, lanes=4, pair_kernel=3), a) == S.OK


@pytest.mark.parametrize("kw, radii, needle", [
    (dict(dt=0.0), None, "dt"),
    (dict(dt=-1e-4), None, "dt"),
    (dict(xi_min=0.05, xi_cut=0.05), None, "xi_min"),
    (dict(xi_min=0.0), None, "xi_min"),
    (dict(mu=-0.1), None, "non-negative"),
    (dict(kT=-1.0), None, "non-negative"),
    (dict(box=(4.4, 20.0, 20.0)), None, "twice the list range"),
    (dict(precision=7), None, "precision"),
    (dict(nlist_cap=65), None, "nlist_cap"),
    (dict(), np.array([1.0, -1.0]), "radius"),
    (dict(), np.array([1.0, 0.0]), "radius"),
    (dict(rho=0.0), None, "rho"),
    (dict(lanes=3), None, "lanes"),
    (dict(lanes=8), None, "lanes"),
    (dict(pair_kernel=4), None, "pair_kernel"),
    (dict(pair_kernel=1), None, "pair_kernel"),
    (dict(pair_kernel=2), None, "pair_kernel"),
    (dict(repulsion=-1.0), None, "non-negative"),
    (dict(cell_factor=0.5), None, "cell_factor"),
    (dict(cell_factor=5.0), None, "cell_factor"),
    # the repulsion reaches a gap of 16 kappa: its list range is 2 * 1.16 + skin
    (dict(box=(5.0, 20.0, 20.0), repulsion=1.0), None, "twice the list range"),
    # a tuned skin must fit with its smallest candidate (0.1 a_min)
    (dict(box=(4.3, 20.0, 20.0), skin=-1.0), None, "twice the list range"),
    (dict(flags=0x400 | 0x800), None, "exclude each other"),
    (dict(flags=0x400, precision=1), None, "SIM_HALF_OCC_ON"),
    (dict(flags=0x400 | 0x20), None, "SIM_HALF_OCC_ON"),
    (dict(flags=0x400, repulsion=1.0), None, "SIM_HALF_OCC_ON"),
])
def test_validate_rejects(kw, radii, needle):
    a = np.full(4, 1.0) if radii is None else radii
    assert S.validate(_cfg(**kw), a) == S.EINVAL
    assert needle in S.last_error()


def test_validate_rejects_struct_size_and_empty():
    c = _cfg().c(3)
    c.struct_size = 8
    a = np.ones(3)
    assert P.lib().sim_validate(C.byref(c), a.ctypes.data_as(C.POINTER(C.c_double))) == S.EINVAL
    c = _cfg().c(0)
    assert P.lib().sim_validate(C.byref(c), a.ctypes.data_as(C.POINTER(C.c_double))) == S.EINVAL


def test_strerror_and_null_handles():
    L = P.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.sim_strerror(code)
    assert L.sim_step(None, 1) == S.EINVAL
    assert L.sim_destroy(None) == S.OK


def test_create_rejects_bad_state_on_the_host():
    """sim_create checks its host inputs before any device work (this runs without a GPU): a coordinate
    outside [0, L), a NaN velocity or an infinite angular velocity is SIM_EINVAL with a message."""
    n = 8
    arr = (S._Config * 1)(_cfg().c(n))
    a = np.full(n, 1.0)
    x = np.random.default_rng(0).random((n, 3)) * 19.0
    v, w = np.zeros((n, 3)), np.zeros((n, 3))

    def ptr(m):
        return (C.POINTER(C.c_double) * 1)(m.ctypes.data_as(C.POINTER(C.c_double)))

    for key, val, needle in (("x", 20.0, "outside [0, L)"), ("x", np.nan, "outside [0, L)"),
                             ("v", np.nan, "velocity value"), ("w", np.inf, "angular velocity value")):
        arrs = dict(x=x.copy(), v=v.copy(), w=w.copy())
        arrs[key][2, 1] = val
        h = C.c_void_p()
        rc = P.lib().sim_create(arr, 1, ptr(a), ptr(arrs["x"]), ptr(arrs["v"]), ptr(arrs["w"]), None, C.byref(h))
        assert rc == S.EINVAL and not h.value
        assert needle in S.last_error(), S.last_error()
