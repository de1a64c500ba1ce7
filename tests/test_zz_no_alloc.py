"""The entry point that allocates nothing: sim_rdf_noalloc, called through the C ABI, against
sim_rdf on the same state, on two calls in a row (the second with fewer bins and a shorter
range, so that stale counts of the first would show), and rejected beyond its array; and its
list build, which leaves a regrow of lists found short to the next call that uses them."""
import ctypes as C
import sys

import numpy as np
import pytest

from inputs import gen

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_rdf_noalloc_matches_rdf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_13802_amd as P
    from paper_2307_13802_amd import sim as S
    L = P.lib()
    st = gen.make_state(gen.Workload("t", 3000, 0.55, 10.0, seed=41))
    # count the library's allocations through the allocator hook
    calls = []

    def _alloc(nbytes, ctx):
        calls.append(int(nbytes))
        return int(torch.cuda.caching_allocator_alloc(int(nbytes)))

    def _free(p, ctx):
        torch.cuda.caching_allocator_delete(p)

    a, f = S._ALLOC_CB(_alloc), S._FREE_CB(_free)
    assert L.sim_set_allocator(a, f, None) == 0
    try:
        sim = P.Sim(P.Config(box=st["L"], **st["params"]), st["radii"], st["x"], st["v"], st["w"])
        sim.step(50)
        for r_max, nb in ((7.5, 3000), (4.0, 37)):
            _say(f"case: sim_rdf_noalloc r_max={r_max} bins={nb}, N=3000")
            before = len(calls)
            got = np.zeros(nb, np.uint64)
            rc = L.sim_rdf_noalloc(sim.h, 0, r_max, nb, got.ctypes.data_as(C.POINTER(C.c_uint64)))
            assert rc == 0, P.sim._err(sim.h)
            assert len(calls) == before   # nothing allocated through the library
            ref = sim.rdf(r_max, nb)      # the allocating entry point on the same state
            assert got.sum() > 1000 and np.array_equal(got, ref)
        bad = np.zeros(70000, np.uint64)
        assert L.sim_rdf_noalloc(sim.h, 0, 4.0, 70000, bad.ctypes.data_as(C.POINTER(C.c_uint64))) == P.sim.EINVAL
        assert "65536" in P.sim._err(sim.h)
        sim.close()
    finally:
        P.use_default_allocator()


def test_rdf_noalloc_leaves_list_regrow_to_next_use():
    """A list build inside sim_rdf_noalloc that finds more partners than the lists hold allocates
    nothing: the lists are regrown by the next call that uses them, and the run stays the run of a
    handle with room for 64 entries (lists and states bit-identical)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_13802_amd as P
    from paper_2307_13802_amd import sim as S
    L = P.lib()
    st = gen.make_state(gen.Workload("t", 300, 0.5, 1.0, kT=1.0, seed=0, mu=0.5))
    big = P.Sim(P.Config(box=st["L"], skin=3.0, lanes=1, nlist_cap=64, **st["params"]), st["radii"], st["x"],
                st["v"], st["w"])
    cap0 = int(np.bincount(big.nlist().reshape(-1), minlength=300).max())
    # the handle under test allocates through a counting hook for its whole life
    calls = []

    def _alloc(nbytes, ctx):
        calls.append(int(nbytes))
        return int(torch.cuda.caching_allocator_alloc(int(nbytes)))

    def _free(p, ctx):
        torch.cuda.caching_allocator_delete(p)

    a, f = S._ALLOC_CB(_alloc), S._FREE_CB(_free)
    assert L.sim_set_allocator(a, f, None) == 0
    grew = False
    try:
        tight = P.Sim(P.Config(box=st["L"], skin=3.0, lanes=1, nlist_cap=cap0, **st["params"]), st["radii"],
                      st["x"], st["v"], st["w"])
        assert tight.stats()["list_cap"] == cap0 and calls
        for k in range(10):
            big.step(200)
            tight.step(200)
            before = tight.stats()["list_cap"]
            n0 = len(calls)
            got = np.zeros(64, np.uint64)
            rc = L.sim_rdf_noalloc(tight.h, 0, 6.0, 64, got.ctypes.data_as(C.POINTER(C.c_uint64)))
            assert rc == 0, P.sim._err(tight.h)
            assert len(calls) == n0   # nothing allocated, even with lists found short
            # the allocating entry point on the other handle: the same histogram, and its lists
            # built from the same positions
            assert np.array_equal(got, big.rdf(6.0, 64))
            after = tight.stats()["list_cap"]   # uses the lists: regrows them if the build left them short
            _say(f"case: step {200 * (k + 1)}: list capacity {before} -> {after} (initial {cap0})")
            assert np.array_equal(tight.nlist(), big.nlist())
            if after > before:
                grew = True
                break
        tight.step(100)
        big.step(100)
        ga, gb = tight.get_state(), big.get_state()
        for key in ("x", "v", "w", "F", "T"):
            assert np.array_equal(ga[key], gb[key]), key
        tight.close()
        big.close()
    finally:
        P.use_default_allocator()
    if not grew:
        pytest.skip(f"no list outgrew its capacity {cap0} in 2000 steps: the deferred regrow was not reached")
