"""The C-ABI library on a machine without a GPU: it loads, exports every entry
point the headers declare, and rejects bad configurations and arguments
before touching HIP (CPU only)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1201_3185_amd", "libqumond.so")


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(qumond_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def Q():
    if not os.path.exists(LIB):
        from paper_1201_3185_amd import build
        build.build()
    from paper_1201_3185_amd import qumond
    return qumond


def test_every_declared_symbol_is_exported(Q):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(qumond_[a-z0-9_]+)\b", out))
    declared = _declared()
    assert len(declared) >= 20
    missing = [d for d in declared if d not in exported]
    assert not missing, missing
    assert set(declared) <= set(Q.exported_symbols())
    Q.lib()  # loads, binds every signature


def test_default_config_is_the_papers(Q):
    c = Q.qumond_config()
    Q.lib().qumond_default_config(ctypes.byref(c))
    assert (c.n, c.nbox, c.npre, c.npost, c.ncycle_fmg) == (65, 1, 2, 2, 6)
    assert c.a0 == 3600.0 and c.gather_frac == 0.2
    assert Q.lib().qumond_validate_config(ctypes.byref(c)) == Q.QUMOND_OK


@pytest.mark.parametrize("change", [
    dict(n=64), dict(n=3), dict(n=2049), dict(box_side=[]), dict(box_side=[100.0, 60.0]),
    dict(box_side=[-1.0]), dict(G=0.0), dict(a0=-1.0), dict(npre=0, npost=0), dict(npre=9),
    dict(ncycle_fmg=0), dict(max_vcycles=-1), dict(tol_rel=-1e-3), dict(precision=7), dict(outer_bc=3),
    dict(gather_frac=0.5), dict(gather_frac=0.0), dict(fixed_shift=-2), dict(nu_n=0.5), dict(nu_n=10.5),
    dict(nu_n=float("nan")),
])
def test_invalid_configs_rejected_without_gpu(Q, change):
    cfg = Q.Config(**change)
    assert Q.validate_config(cfg) == Q.QUMOND_ERR_INVALID
    c = cfg.to_c()
    h = ctypes.c_void_p()
    assert Q.lib().qumond_create(ctypes.byref(c), None, ctypes.byref(h)) == Q.QUMOND_ERR_INVALID
    assert not h.value
    assert len(Q.lib().qumond_last_error()) > 0


def test_valid_nested_configs(Q):
    assert Q.validate_config(Q.Config(n=129, box_side=[400.0, 200.0, 100.0, 50.0])) == Q.QUMOND_OK
    assert Q.validate_config(Q.Config(n=5, box_side=[1.0])) == Q.QUMOND_OK
    assert Q.validate_config(Q.Config(n=513, box_side=[120.0], precision=Q.QUMOND_MIXED)) == Q.QUMOND_OK
    assert Q.validate_config(Q.Config(nu_n=2.0)) == Q.QUMOND_OK
    c = Q.qumond_config()
    Q.lib().qumond_default_config(ctypes.byref(c))
    assert c.nu_n == 1.0


def test_null_handles_and_arguments(Q):
    L = Q.lib()
    assert L.qumond_destroy(None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_deposit(None, None, None, None, None, 0, 1.0, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_solve_newton(None, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_mond_source(None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_solve_mond(None, None, 0, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_gather_forces(None, None, None, None, 0, 0, None, None, None, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_k_rbgs_sweep(64, 1.0, None, None, None, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_k_rbgs_sweep_from_zero(33, 1.0, None, None, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_k_rbgs_sweep_from_zero(34, 1.0, None, None, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_k_fmg(33, 1.0, None, None, 2, 2, 6, 0, 0.0, None, None, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_status_string(Q.QUMOND_ERR_STATE) == b"call out of order"


def test_split_prolong_table_without_gpu(Q):
    for n in (33, 129):
        before = Q.tune_get_split(n)
        Q.tune_set_split(n, 1 - before)
        assert Q.tune_get_split(n) == 1 - before and Q.tune_get_split(n, fp32=True) in (0, 1)
        Q.tune_set_split(n, before)
    L = Q.lib()
    assert L.qumond_tune_set_split(33, 0, 2) == Q.QUMOND_ERR_INVALID
    assert L.qumond_tune_set_split(34, 0, 1) == Q.QUMOND_ERR_INVALID
    assert L.qumond_tune_get_split(33, 0, None) == Q.QUMOND_ERR_INVALID


# ------------------------------------------------------------ batches

def _batch_args(Q, cfg, ns, R):
    c = cfg.to_c(len(ns))
    return c, (ctypes.c_int32 * len(ns))(*ns), (ctypes.c_double * max(1, len(R)))(*R)


def test_batch_defaults(Q):
    c = Q.qumond_batch_config()
    Q.lib().qumond_batch_default_config(ctypes.byref(c))
    assert (c.npre, c.npost, c.ncycle_fmg, c.refine_iters, c.naz) == (2, 2, 2, 4, 16)
    assert c.tol_rel == 1e-6 and c.box_side == 120.0 and c.a0 == 3600.0
    assert Q.batch_validate(Q.BatchConfig(), [129, 257, 129], [1.0, 2.0]) == Q.QUMOND_OK


@pytest.mark.parametrize("ns,R,change", [
    ([130], [1.0], {}), ([9], [1.0], {}), ([2049], [1.0], {}), ([129], [], {}), ([129], [-1.0], {}),
    ([129], [float("nan")], {}), ([257] * 600, [1.0], {}), ([129], [1.0], dict(box_side=0.0)),
    ([129], [1.0], dict(G=-1.0)), ([129], [1.0], dict(npre=0, npost=0)), ([129], [1.0], dict(ncycle_fmg=0)),
    ([129], [1.0], dict(refine_iters=-1)), ([129], [1.0], dict(max_extra=-1)), ([129], [1.0], dict(tol_rel=-1.0)),
    ([129], [1.0], dict(gather_frac=0.6)), ([129], [1.0], dict(naz=0)), ([129], [1.0], dict(nu_n=0.9)),
])
def test_batch_invalid_rejected_without_gpu(Q, ns, R, change):
    cfg = Q.BatchConfig(**change)
    c, nn, rr = _batch_args(Q, cfg, ns, R)
    assert Q.lib().qumond_batch_validate(ctypes.byref(c), nn, rr if R else None, len(R)) == Q.QUMOND_ERR_INVALID
    h = ctypes.c_void_p()
    assert Q.lib().qumond_batch_create(ctypes.byref(c), nn, rr if R else None, len(R), None,
                                       ctypes.byref(h)) == Q.QUMOND_ERR_INVALID
    assert not h.value and len(Q.lib().qumond_last_error()) > 0


def test_batch_null_handles(Q):
    L = Q.lib()
    assert L.qumond_batch_destroy(None) == Q.QUMOND_OK
    assert L.qumond_batch_run(None, 1, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_batch_set_particles(None, 0, None, None, None, None, 0, 1.0) == Q.QUMOND_ERR_INVALID
    assert L.qumond_batch_rotation_curves(None, 1, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_batch_get_field(None, 0, Q.FIELD_PHI, None) == Q.QUMOND_ERR_INVALID
    assert L.qumond_batch_device_bytes(None) == 0
    c = Q.BatchConfig().to_c(1)
    assert L.qumond_batch_validate(ctypes.byref(c), None, None, 0) == Q.QUMOND_ERR_INVALID


def test_tune_tables_keep_entries_of_both_precisions():
    """Setting a launch shape for one precision never resets the other's
    table (the defaults are written once for both), so the entries of a
    loaded table survive whatever order its FP64 and FP32 rows come in; the
    correcting sweep's shape defaults to the plain sweep's (-1), is set per
    precision and is read from a table.  Run in a fresh process: the first
    use of each precision's table is the case."""
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1201_3185_amd import qumond as Q\n"
        "Q.tune_set_fused(33, 3, 0, fp32=False)\n"
        "Q.tune_set(33, 9, 0, fp32=False)\n"
        "Q.tune_set_fused(33, 4, 0, fp32=True)\n"
        "Q.tune_set(33, 10, 0, fp32=True)\n"
        "assert Q.tune_get_fused(33, fp32=False) == (3, 0), Q.tune_get_fused(33, fp32=False)\n"
        "assert Q.tune_get(33, fp32=False) == (9, 0)\n"
        "assert Q.tune_get_fused(33, fp32=True) == (4, 0)\n"
        "assert Q.tune_get(33, fp32=True) == (10, 0)\n"
        "assert Q.tune_get_corr(65, fp32=False) == (-1, 0)\n"
        "Q.tune_set_corr(65, 13, 32, fp32=False)\n"
        "assert Q.tune_get_corr(65, fp32=False) == (13, 32) and Q.tune_get_corr(65, fp32=True) == (-1, 0)\n"
        "import json, tempfile\n"
        "t = tempfile.NamedTemporaryFile('w', suffix='.json', delete=False)\n"
        "json.dump({'smoother': [{'n': 129, 'fp32': 1, 'corr_variant': 11, 'corr_kchunk': 8, 'us': 1.0}]}, t)\n"
        "t.close()\n"
        "Q.tune_load(t.name)\n"
        "assert Q.tune_get_corr(129, fp32=True) == (11, 8)\n"
        "assert Q.tune_get_corr(65, fp32=False) == (13, 32)\n"
        "assert Q.tune_get_sweep_restrict(257) == 0\n"
        "Q.tune_set_sweep_restrict(257, 1)\n"
        "assert Q.tune_get_sweep_restrict(257) == 1 and Q.tune_get_sweep_restrict(257, fp32=True) == 0\n"
        "t2 = tempfile.NamedTemporaryFile('w', suffix='.json', delete=False)\n"
        "json.dump({'smoother': [{'n': 513, 'fp32': 1, 'sweep_restrict': 1, 'us': [2.0, 1.0]}]}, t2)\n"
        "t2.close()\n"
        "Q.tune_load(t2.name)\n"
        "assert Q.tune_get_sweep_restrict(513, fp32=True) == 1\n"
        "try:\n"
        "    Q.tune_set_corr(65, 99, 0)\n"
        "    raise SystemExit('bad variant accepted')\n"
        "except Q.QumondError:\n"
        "    pass\n"
        "print('ok')\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
