"""The coarse-grid correction of a V-cycle (u += P uc before post-smoothing)
runs either inside the first post-smoothing launch or as a prolong-add launch
of its own; the autotuner picks per level and precision.  Both forms must give
the same bits, in the FP64 and mixed solvers (eager and graph replay) and in
the batched runner over stacked problems."""
import numpy as np
import pytest
import torch

from paper_1201_3185_amd import qumond as Q
from paper_1201_3185_amd import synth

pytestmark = pytest.mark.gpu

LEVELS = (33, 65, 129)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def set_all(split):
    for n in LEVELS:
        for fp in (False, True):
            Q.tune_set_split(n, split, fp32=fp)


@pytest.fixture
def saved_split():
    saved = {(n, fp): Q.tune_get_split(n, fp32=fp) for n in LEVELS for fp in (False, True)}
    yield
    for (n, fp), v in saved.items():
        Q.tune_set_split(n, v, fp32=fp)


@pytest.mark.parametrize("precision,graphs", [(Q.QUMOND_FP64, 0), (Q.QUMOND_FP64, 1), (Q.QUMOND_MIXED, 0)])
def test_context_split_is_bitwise_identical(saved_split, precision, graphs):
    p = synth.two_component_disk(20000, synth.seed_for(5, 11))
    out = []
    for split in (0, 1):
        set_all(split)
        assert all(Q.tune_get_split(n) == split for n in LEVELS)
        ctx = Q.Context(Q.Config(n=129, box_side=[100.0, 50.0], precision=precision, use_graphs=graphs,
                                 tol_rel=1e-8))
        ctx.deposit(dev(p.x), dev(p.y), dev(p.z), dev(p.m), p.total_mass)
        i_n, i_m = ctx.solve()
        if graphs:   # a second solve replays the captured schedules
            i_n, i_m = ctx.solve()
        out.append(([ctx.get_field(b, f).cpu().numpy() for b in range(2) for f in (Q.FIELD_PHI_N, Q.FIELD_PHI)],
                    i_n["vcycles"], i_m["vcycles"]))
        ctx.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    assert out[0][1:] == out[1][1:]


def test_batch_split_is_bitwise_identical(saved_split):
    ns = [65, 129, 33, 65]
    parts = [synth.two_component_disk(15000 + 1000 * i, synth.seed_for(6, 20 + i)) for i in range(len(ns))]
    fields = []
    for split in (0, 1):
        set_all(split)
        b = Q.Batch(Q.BatchConfig(box_side=120.0, refine_iters=3, tol_rel=1e-300, max_extra=0), ns,
                    [1.0, 5.0, 20.0])
        for i, pp in enumerate(parts):
            b.set_particles(i, dev(pp.x), dev(pp.y), dev(pp.z), dev(pp.m), pp.total_mass)
        b.run(use_graph=split == 1, allow_not_converged=True)
        fields.append([b.get_field(i, Q.FIELD_PHI).cpu().numpy() for i in range(len(ns))])
        b.close()
    for a, c in zip(*fields):
        assert np.array_equal(a, c)
