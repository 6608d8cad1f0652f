"""The oracle's node-parallel loops give the same bits at any thread count.

Only loops whose iterations write distinct nodes and read nothing another
iteration writes run on several threads (a colour pass of red-black
Gauss-Seidel, residual, restriction, prolongation, interpolation, the Eq. 2
source, the per-point gather); the deposit and every sum stay serial.  So the
whole pipeline -- density, both potentials, the source, forces and V-cycle
counts -- must be identical with one thread and with several.
"""
import numpy as np

import oracle as O
from paper_1201_3185_amd import synth


def _pipeline(threads):
    prev = O.set_threads(threads)
    try:
        p = synth.two_component_disk(20000, synth.seed_for(3, 41))
        oc = O.OracleConfig(n=33, box_side=[100.0, 50.0], tol_rel=1e-10)
        r = O.run_pipeline(oc, p.x, p.y, p.z, p.m, p.total_mass)
        g = O.gather(r.phi, oc.box_side, p.x[:3000], p.y[:3000], p.z[:3000], M=p.total_mass, mond=True)
    finally:
        O.set_threads(prev)
    return r, g


def test_pipeline_is_bitwise_independent_of_threads():
    r1, g1 = _pipeline(1)
    r4, g4 = _pipeline(4)
    for b in range(2):
        for a, c in ((r1.q, r4.q), (r1.f, r4.f), (r1.phin, r4.phin), (r1.S, r4.S), (r1.phi, r4.phi)):
            assert np.array_equal(a[b], c[b])
    assert r1.info_newton == r4.info_newton and r1.info_mond == r4.info_mond
    for a, c in zip(g1, g4):
        assert np.array_equal(a, c)
    # the schedule really iterated (not a trivial comparison)
    assert all(info[2] >= 1 for info in r1.info_newton)


def test_thread_count_is_restored():
    prev = O.set_threads(3)
    assert O.set_threads(prev) == 3
