"""The allocation-free residual norms (qumond_k_resid_norms_noalloc) give the
bits of qumond_k_resid_norms, the entry point it mirrors, through the C ABI:
two calls in a row, the second on a smaller grid (so the shared workspace
holds the first call's partial sums when the second starts), and a grid
beyond the workspace maximum is refused before any launch."""
import numpy as np
import pytest
import torch

from paper_1201_3185_amd import qumond as Q

pytestmark = pytest.mark.gpu


def _noalloc(f, u, h, out):
    return Q.lib().qumond_k_resid_norms_noalloc(int(u.shape[0]), float(h), f.data_ptr(), u.data_ptr(),
                                                 out.data_ptr(), torch.cuda.current_stream().cuda_stream)


def _state(n, seed):
    rng = np.random.default_rng(seed)
    f = torch.from_numpy(rng.standard_normal((n, n, n))).cuda()
    u = torch.from_numpy(rng.standard_normal((n, n, n))).cuda()
    return f, u


def test_noalloc_norms_match_allocating_entry_point():
    for n, seed in ((257, 11), (33, 12)):            # the second call on a smaller grid
        f, u = _state(n, seed)
        h = 7.0 / (n - 1)
        ref = torch.zeros(3, dtype=torch.float64, device="cuda")
        Q.k_resid_norms(f, u, h, ref)
        got = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
        assert _noalloc(f, u, h, got) == Q.QUMOND_OK
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy()), n
        assert (got.cpu().numpy() > 0).all()


def test_noalloc_refuses_grid_beyond_workspace():
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = Q.lib().qumond_k_resid_norms_noalloc(2049, 1.0, t.data_ptr(), t.data_ptr(), t.data_ptr(), None)
    assert st == Q.QUMOND_ERR_INVALID
    assert b"workspace maximum" in Q.lib().qumond_last_error()
