"""MI355X (gfx950) Triad-ATRG coarse-graining for the 4D Ising model.

Thin ctypes binding of libtatrg.so (include/tatrg.h, include/tatrg_testing.h): argument
marshalling only.  Every step of the RG runs in the library's HIP kernels; PyTorch is used
for device memory and the stream.  Importing this package without the built library raises.
"""
import ctypes
import os

__all__ = ["lib", "TatrgConfig", "Engine", "TatrgError", "FP64", "BF16X3", "library_path"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libtatrg.so")

FP64 = 0
BF16X3 = 1

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENUMERIC", -5: "ESTATE"}


class TatrgError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, msg))
        self.status = status


def _load():
    if not os.path.exists(library_path):
        raise ImportError("libtatrg.so is not built; run python paper_2412_14104_amd/build.py")
    # torch (which owns the device memory and streams handed to the library) is imported
    # first, so its HIP runtime is initialised before the library's; loading the library
    # first leaves the library's runtime without a device
    import torch  # noqa: F401
    return ctypes.CDLL(library_path)


lib = _load()


class TatrgConfig(ctypes.Structure):
    _fields_ = [("chi", ctypes.c_int32), ("r", ctypes.c_int32), ("q", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("record_spectra", ctypes.c_int32), ("swap_mode", ctypes.c_int32)]


_p = ctypes.c_void_p
_i32, _i64, _u32, _u64, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
_cfgp = ctypes.POINTER(TatrgConfig)
_dblp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "tatrg_workspace_bytes": (ctypes.c_size_t, [_cfgp]),
    "tatrg_create": (ctypes.c_int, [_cfgp, _p, ctypes.c_size_t, _p, ctypes.POINTER(_p)]),
    "tatrg_init_tensor": (ctypes.c_int, [_p, _dblp]),
    "tatrg_step": (ctypes.c_int, [_p]),
    "tatrg_rsvd": (ctypes.c_int, [_p, _p, _i64, _i64, _i64, _i32, _i32, _i32, _u64, _u32, _p,
                                  _p, _p]),
    "tatrg_rsvd_noalloc": (ctypes.c_int, [_p, _i64, _i64, _i64, _i32, _i32, _i32, _u64, _u32,
                                          _p, _p, _p, _p]),
    "tatrg_lognorm": (ctypes.c_int, [_p, _dblp]),
    "tatrg_free_energy": (ctypes.c_int, [_p, _dblp, _dblp]),
    "tatrg_lnz_derivatives": (ctypes.c_int, [_p, _dblp, _dblp, _dblp]),
    "tatrg_set_side_stream": (ctypes.c_int, [_p, _i32]),
    "tatrg_autotune": (ctypes.c_int, [_p, ctypes.POINTER(_i32)]),
    "tatrg_get_spectra": (ctypes.c_int, [_p, _i32, _i32, _dblp, _i32, ctypes.POINTER(_i32)]),
    "tatrg_get_record": (ctypes.c_int, [_p, _i32, _i32, _i32, _dblp, _i32,
                                        ctypes.POINTER(_i32)]),
    "tatrg_get_state": (ctypes.c_int, [_p, _p, _p, ctypes.POINTER(_i32), _dblp]),
    "tatrg_set_state": (ctypes.c_int, [_p, _p, _p, _i32, _dbl]),
    "tatrg_last_error": (ctypes.c_char_p, [_p]),
    "tatrg_destroy": (None, [_p]),
    "tatrg_test_gemm": (ctypes.c_int, [_p, _p, _p, _i64, _i64, _i64, _i64, _i64, _i64,
                                       ctypes.c_int, ctypes.c_int, _dbl, _dbl, _i64, _i64,
                                       _i64, _i64, ctypes.c_int, _p, _p]),
    "tatrg_test_gemm_bf16x3_ws": (ctypes.c_size_t, [_i64, _i64, _i64, _i64, _i64,
                                                    ctypes.c_int, ctypes.c_int, _i64, _i64,
                                                    _i64]),
    "tatrg_test_gemm_bf16x3": (ctypes.c_int, [_p, _p, _p, _i64, _i64, _i64, _i64, _i64, _i64,
                                              ctypes.c_int, ctypes.c_int, _dbl, _dbl, _i64,
                                              _i64, _i64, _i64, _p, _p]),
    "tatrg_test_gemm_bf16x3_chain_ws": (ctypes.c_size_t, [_i64] * 6),
    "tatrg_test_gemm_bf16x3_chain": (ctypes.c_int, [_p, _p, _p, _p] + [_i64] * 6 +
                                     [_p, ctypes.c_size_t, _p]),
    "tatrg_test_split_products": (ctypes.c_int, [ctypes.c_int]),
    "tatrg_test_tsqr_ws": (ctypes.c_size_t, [_i64, ctypes.c_int]),
    "tatrg_test_tsqr": (ctypes.c_int, [_p, _i64, ctypes.c_int, _i64, _p, _p, _p]),
    "tatrg_test_svd": (ctypes.c_int, [_p, _p, _p, _p, ctypes.c_int, ctypes.c_int, _p]),
    "tatrg_test_cholesky": (ctypes.c_int, [_p, ctypes.c_int, ctypes.c_int, _dbl, _p, _p]),
    "tatrg_test_cholesky_blocked_inv": (ctypes.c_int, [_p, _p, _p, _p, ctypes.c_int,
                                                       ctypes.c_int, _p, _p]),
    "tatrg_test_chol_inv": (ctypes.c_int, [_p, _p, _p, ctypes.c_int, ctypes.c_int, _dbl, _p,
                                            _p]),
    "tatrg_test_chol_inv_batched": (ctypes.c_int, [_p, _p, _p, ctypes.c_int, ctypes.c_int, _dbl,
                                                   _p, ctypes.c_int, _p]),
    "tatrg_test_philox": (ctypes.c_int, [_p, _i64, _i64, _u64, _u32, _u32, _p]),
    "tatrg_test_philox_words": (ctypes.c_int, [_p, _i64, _i64, _u64, _u32, _u32, _p]),
    "tatrg_test_permute": (ctypes.c_int, [_p, _p, ctypes.c_int, ctypes.POINTER(_i64),
                                          ctypes.POINTER(ctypes.c_int), _p]),
    "tatrg_test_gauge": (ctypes.c_int, [_p, _p, _p, ctypes.c_int, ctypes.c_int, _dbl, _dbl,
                                        _p]),
    "tatrg_profile_enable": (ctypes.c_int, [_p, ctypes.c_int]),
    "tatrg_profile_read": (ctypes.c_int, [_p, _dblp, ctypes.POINTER(_i32), _dblp]),
    "tatrg_test_speculation": (ctypes.c_int, [_p, ctypes.c_int, ctypes.POINTER(_i64)]),
    "tatrg_profile_read_stages": (ctypes.c_int, [_p, _dblp, ctypes.POINTER(_i32)]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def _check(status, handle=None):
    if status != 0:
        msg = lib.tatrg_last_error(handle).decode() if handle else ""
        raise TatrgError(status, msg)


def _stream_ptr(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


class Engine:
    """One RG run (or a batch of `batch` temperatures sharing the sketches) on the current HIP
    device.  The workspace is a torch uint8 tensor on the device; the stream is torch's
    current stream unless one is given."""

    def __init__(self, chi, r, q, n_steps, seed=0, precision=FP64, record_spectra=True,
                 stream=None, device="cuda", batch=1, swap_mode=0):
        import torch
        self.cfg = TatrgConfig(chi=chi, r=r, q=q, n_steps=n_steps, batch=batch,
                               precision=precision, seed=seed,
                               record_spectra=1 if record_spectra else 0,
                               swap_mode=swap_mode)
        nbytes = lib.tatrg_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise TatrgError(-1, "invalid configuration")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.handle = ctypes.c_void_p()
        _check(lib.tatrg_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.ws.data_ptr()),
                                nbytes, _stream_ptr(self.stream), ctypes.byref(self.handle)))
        self.chi, self.n_steps, self.batch = chi, n_steps, batch

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:  # lib is None at interpreter exit
            lib.tatrg_destroy(h)
            self.handle = None

    def init(self, beta):
        """beta: one value (batch 1) or a sequence of `batch` values."""
        betas = [beta] if isinstance(beta, (int, float)) else list(beta)
        if len(betas) != self.batch:
            raise TatrgError(-1, "need %d temperatures" % self.batch)
        arr = (ctypes.c_double * self.batch)(*betas)
        _check(lib.tatrg_init_tensor(self.handle, arr), self.handle)

    def step(self):
        _check(lib.tatrg_step(self.handle), self.handle)

    def lognorm(self):
        out = (ctypes.c_double * self.batch)()
        _check(lib.tatrg_lognorm(self.handle, out), self.handle)
        return out[0] if self.batch == 1 else list(out)

    def free_energy(self):
        """(f, ln Z / V): floats for batch 1, lists of `batch` values otherwise."""
        f = (ctypes.c_double * self.batch)()
        lnzv = (ctypes.c_double * self.batch)()
        _check(lib.tatrg_free_energy(self.handle, f, lnzv), self.handle)
        if self.batch == 1:
            return f[0], lnzv[0]
        return list(f), list(lnzv)

    def set_side_stream(self, on):
        """Run the step's independent work on the handle's second stream (default) or, with
        on=False, in order on its own stream; results are bit for bit the same."""
        _check(lib.tatrg_set_side_stream(self.handle, 1 if on else 0), self.handle)

    def autotune(self):
        """Measured work-group grouping of the split GEMMs (tatrg_autotune): the three
        chosen values, or -1 each on the FP64 path."""
        out = (_i32 * 3)()
        _check(lib.tatrg_autotune(self.handle, out), self.handle)
        return list(out)

    def lnz_derivatives(self):
        """For a batch of triples (beta - d, beta, beta + d): lists (ln Z/V, d(ln Z/V)/d beta,
        d^2(ln Z/V)/d beta^2) of batch / 3 entries (tatrg_lnz_derivatives)."""
        n = self.batch // 3
        l0, d1, d2 = ((ctypes.c_double * max(n, 1))() for _ in range(3))
        _check(lib.tatrg_lnz_derivatives(self.handle, l0, d1, d2), self.handle)
        return list(l0[:n]), list(d1[:n]), list(d2[:n])

    def spectrum(self, step, which, b=0):
        buf = (ctypes.c_double * self.chi)()
        n = ctypes.c_int32()
        _check(lib.tatrg_get_record(self.handle, b, step, which, buf, self.chi,
                                    ctypes.byref(n)), self.handle)
        return [buf[i] for i in range(n.value)]

    def swap_compressed(self, step, b=0):
        """1 when the bond swap of `step` ran on the compressed cell middle, 0 on the full
        one, -1 when the step has not run."""
        buf = (ctypes.c_double * 1)()
        n = ctypes.c_int32()
        _check(lib.tatrg_get_record(self.handle, b, step, 6, buf, 1, ctypes.byref(n)),
               self.handle)
        return int(buf[0])

    def order_parameter(self, step, b=0):
        """X^(step) of temperature b (recorded with record_spectra)."""
        return self.spectrum(step, 5, b)[0]

    def get_state(self, phi, psi):
        step, acc = ctypes.c_int32(), ctypes.c_double()
        _check(lib.tatrg_get_state(self.handle, ctypes.c_void_p(phi.data_ptr()),
                                   ctypes.c_void_p(psi.data_ptr()), ctypes.byref(step),
                                   ctypes.byref(acc)), self.handle)
        return step.value, acc.value

    def set_state(self, phi, psi, step, acc):
        _check(lib.tatrg_set_state(self.handle, ctypes.c_void_p(phi.data_ptr()),
                                   ctypes.c_void_p(psi.data_ptr()), step, acc), self.handle)

    def profile_enable(self, max_launches):
        _check(lib.tatrg_profile_enable(self.handle, max_launches), self.handle)

    def profile_read(self):
        """(summed device ms, launches, flops per launch) of the timed contraction GEMMs."""
        ms, n, fl = ctypes.c_double(), ctypes.c_int32(), ctypes.c_double()
        _check(lib.tatrg_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n),
                                      ctypes.byref(fl)), self.handle)
        return ms.value, n.value, fl.value

    def profile_read_stages(self):
        """(summed device ms of stages S0..S5 as a list of six, steps timed)."""
        ms = (ctypes.c_double * 6)()
        n = ctypes.c_int32()
        _check(lib.tatrg_profile_read_stages(self.handle, ms, ctypes.byref(n)), self.handle)
        return list(ms), n.value

    def run(self, beta):
        """All n_steps steps; returns (f, ln Z / V)."""
        self.init(beta)
        for _ in range(self.n_steps):
            self.step()
        return self.free_energy()


def run(beta, chi, r, q, n_steps, seed=0, record_spectra=False):
    """Convenience: free energy per site and ln Z / V of one run."""
    eng = Engine(chi, r, q, n_steps, seed=seed, record_spectra=record_spectra)
    f, lnzv = eng.run(beta)
    return {"f": f, "lnZV": lnzv, "engine": eng}

