"""Thin ctypes binding of libblochwave.so (the C ABI in include/blochwave.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device vectors are torch tensors (complex128 for BW_FP64 cells,
complex64 for BW_MIXED cells) of shape (nvec, 3, n0, n1, n2), contiguous, on
the current HIP device; the current torch stream is used unless one is given.
The library must be built (``python -m paper_2106_12487_amd.build_lib``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblochwave.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "blochwave.h")

BW_OK, BW_ENOTCONV, BW_ESTALL = 0, 1, 2
BW_EINVAL, BW_ENOMEM, BW_EHIP, BW_EUNSUPPORTED = -1, -2, -3, -4
BW_FP64, BW_MIXED = 0, 1
BW_SUBSPACE, BW_LANCZOS = 0, 1
BW_PLAIN, BW_LEARNED = 0, 1


class BlochwaveError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"blochwave error {code}: {msg}")
        self.code = code


class bw_eig_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("block", ctypes.c_int32), ("ncv", ctypes.c_int32),
                ("maxit_outer", ctypes.c_int32), ("maxit_lin", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("tol_eig", ctypes.c_double),
                ("tol_lin", ctypes.c_double), ("tol_omega", ctypes.c_double), ("kbatch", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("net", ctypes.c_void_p), ("group_cells", ctypes.c_int32),
                ("kgroups", ctypes.c_int32)]


class bw_stats(ctypes.Structure):
    _fields_ = [("pcg_iterations", ctypes.c_int64), ("block_iterations", ctypes.c_int64),
                ("outer_iterations", ctypes.c_int64), ("k_applies", ctypes.c_int64),
                ("m_applies", ctypes.c_int64), ("seconds", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "bw_create_rve": (_I, [ctypes.POINTER(_P), _IP, _DP, ctypes.POINTER(ctypes.c_uint16), _I, _DP, _DP, _I, _P]),
    "bw_destroy_rve": (None, [_P]),
    "bw_rve_info": (_I, [_P, _IP, _IP, _DP, _DP]),
    "bw_apply_K": (_I, [_P, _DP, _P, _P, _I, _P]),
    "bw_apply_K_noalloc": (_I, [_P, _DP, _P, _P, _I, _P]),
    "bw_apply_M": (_I, [_P, _P, _P, _I, _P]),
    "bw_apply_P": (_I, [_P, _DP, _P, _P, _I, _P]),
    "bw_pcg_solve": (_I, [_P, _DP, _P, _P, _I, _D, _I, _IP, _DP, _P]),
    "bw_lowest_modes": (_I, [_P, _DP, _I, _I, ctypes.POINTER(bw_eig_opts), _DP, _DP, _P,
                             ctypes.POINTER(bw_stats), _P]),
    "bw_lowest_modes_batched": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_DP), _IP, _I, ctypes.POINTER(bw_eig_opts),
                                     ctypes.POINTER(_DP), ctypes.POINTER(_DP), ctypes.POINTER(_P),
                                     ctypes.POINTER(bw_stats), _P]),
    "bw_last_error": (ctypes.c_char_p, []),
    "bw_timing_enable": (_I, [_I]),
    "bw_timing_report": (ctypes.c_int64, [ctypes.c_char_p, ctypes.c_int64]),
    "bw_timing_filter": (_I, [ctypes.c_char_p]),
    "bw_graphs_enable": (_I, [_I]),
    "bw_autotune": (_I, [_P, _I, _DP, _P]),
    "bw_fft_schedule": (_I, [_P, _IP, _IP, _I]),
    "bw_diag_copy": (_I, [_P, _P, ctypes.c_int64, _P]),
    "bw_unet_param_count": (ctypes.c_int64, []),
    "bw_unet_create": (_I, [ctypes.POINTER(_P), ctypes.c_uint64]),
    "bw_unet_destroy": (None, [_P]),
    "bw_unet_get_weights": (_I, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "bw_unet_set_weights": (_I, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "bw_unet_net_forward": (_I, [_P, _IP, _P, _P, _I, _P]),
    "bw_unet_net_backward": (_I, [_P, _IP, _P, _P, ctypes.POINTER(ctypes.c_float), _I, _P]),
    "bw_unet_apply": (_I, [_P, _P, _DP, _P, _P, _I, _P]),
    "bw_unet_train_step": (_I, [_P, _P, _DP, _P, _P, _I, _D, _DP, _P]),
    "bw_unet_train_step_residual": (_I, [_P, _P, _DP, _P, _I, _D, _DP, _P]),
    "bw_pcg_solve_learned": (_I, [_P, _P, _DP, _P, _P, _I, _D, _I, _IP, _DP, _IP, _P]),
    "bw_group_velocity": (_I, [_P, _DP, _DP, _I, _P, _DP, _D, _DP, _P]),
    "bw_long_wave_speeds": (_I, [_P, _DP, _D, _D, _DP, _P]),
    "bw_mode_fields": (_I, [_P, _DP, _I, _P, _P, _P, _DP, _P]),
    "bw_effective_stiffness": (_I, [_P, ctypes.c_double, _I, _DP, _IP, _P]),
}


def header_symbols() -> list[str]:
    """Function names declared in include/blochwave.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(bw_\w+)\s*\(", txt, flags=re.M)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2106_12487_amd.build_lib`")
        # torch ships its own HIP runtime under the same soname; load it first so
        # that the library and torch share one runtime (device memory, streams).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def bw_last_error() -> str:
    return lib().bw_last_error().decode()


def bw_timing_enable(enable: bool) -> None:
    lib().bw_timing_enable(int(bool(enable)))


def bw_graphs_enable(enable: bool) -> None:
    lib().bw_graphs_enable(int(bool(enable)))


def bw_timing_filter(name) -> None:
    lib().bw_timing_filter(name.encode() if name else None)


def bw_timing_report() -> dict:
    import json
    need = lib().bw_timing_report(None, 0)
    buf = ctypes.create_string_buffer(int(need) + 16)
    lib().bw_timing_report(buf, len(buf))
    return json.loads(buf.value.decode())


def bw_diag_copy(src, dst, stream=None) -> None:
    """Plain device copy of src into dst (same byte size), the counter-calibration kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    _check(lib().bw_diag_copy(_dptr(src), _dptr(dst), nbytes, _stream(stream)))


def _check(code: int) -> int:
    if code < 0:
        raise BlochwaveError(code, bw_last_error())
    return code


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    if not t.is_contiguous():
        raise ValueError("device tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _darr(a) -> ctypes.Array:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_DP)


class Rve:
    """Owning wrapper of a bw_rve handle."""

    def __init__(self, n, L, grain_map, C21, rho, precision: int = BW_FP64, stream=None):
        n_arr = (ctypes.c_int32 * 3)(*[int(v) for v in n])
        L_arr, L_p = _darr(L)
        g = np.ascontiguousarray(grain_map, dtype=np.uint16).reshape(-1)
        C_arr, C_p = _darr(np.asarray(C21).reshape(-1, 21))
        r_arr, r_p = _darr(np.asarray(rho).reshape(-1))
        h = ctypes.c_void_p()
        _check(lib().bw_create_rve(ctypes.byref(h), n_arr, L_p, g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                   int(C_arr.shape[0]), C_p, r_p, int(precision),
                                   _stream(stream) if stream is not None else None))
        self.handle = h
        self.n = tuple(int(v) for v in n)
        self.precision = int(precision)

    @classmethod
    def from_inputs(cls, rve, precision: int = BW_FP64):
        return cls(rve.n, rve.L, rve.grain_map, rve.C21, rve.rho, precision)

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.precision == BW_FP64 else torch.complex64

    def info(self) -> dict:
        n = (ctypes.c_int32 * 3)()
        prec = ctypes.c_int32()
        c0 = (ctypes.c_double * 21)()
        rb = ctypes.c_double()
        _check(lib().bw_rve_info(self.handle, n, ctypes.byref(prec), c0, ctypes.byref(rb)))
        return dict(n=tuple(n), precision=prec.value, C0=np.array(c0[:]), rho_bar=rb.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().bw_destroy_rve(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bw_autotune(rve: Rve, nvec: int = 8, stream=None) -> float:
    """Pick the fastest FFT schedule of the cell by timing; returns the speedup over the default."""
    sp = ctypes.c_double()
    _check(lib().bw_autotune(rve.handle, int(nvec), ctypes.byref(sp), _stream(stream)))
    return sp.value


def bw_fft_schedule(rve: Rve, reg=None, cap=None):
    """Get the cell's FFT schedule (reg, cap), or set it when both are given."""
    r = (ctypes.c_int32 * 3)(*(reg if reg is not None else (0, 0, 0)))
    c = (ctypes.c_int32 * 3)(*(cap if cap is not None else (0, 0, 0)))
    _check(lib().bw_fft_schedule(rve.handle, r, c, int(reg is not None and cap is not None)))
    return list(r), list(c)


def bw_apply_K(rve: Rve, k, u, y, stream=None) -> None:
    k_arr, k_p = _darr(k)
    _check(lib().bw_apply_K(rve.handle, k_p, _dptr(u), _dptr(y), int(u.shape[0]), _stream(stream)))


def bw_apply_K_noalloc(rve: Rve, k, u, y, stream=None) -> None:
    """y = K(k) u with no device allocation (library scratch area; see the header)."""
    k_arr, k_p = _darr(np.asarray(k, dtype=np.float64).reshape(3))
    _check(lib().bw_apply_K_noalloc(rve.handle, k_p, _dptr(u), _dptr(y), int(u.shape[0]), _stream(stream)))


def bw_apply_M(rve: Rve, u, y, stream=None) -> None:
    _check(lib().bw_apply_M(rve.handle, _dptr(u), _dptr(y), int(u.shape[0]), _stream(stream)))


def bw_apply_P(rve: Rve, k, u, y, stream=None) -> None:
    k_arr, k_p = _darr(k)
    _check(lib().bw_apply_P(rve.handle, k_p, _dptr(u), _dptr(y), int(u.shape[0]), _stream(stream)))


def bw_pcg_solve(rve: Rve, k, b, x, rtol: float, maxit: int = 0, stream=None):
    """Solve K(k) x = b in place of x; returns (status, iterations, true relative residuals)."""
    nrhs = int(b.shape[0])
    k_arr, k_p = _darr(k)
    it = np.zeros(nrhs, dtype=np.int32)
    rr = np.zeros(nrhs)
    code = _check(lib().bw_pcg_solve(rve.handle, k_p, _dptr(b), _dptr(x), nrhs, float(rtol), int(maxit),
                                     it.ctypes.data_as(_IP), rr.ctypes.data_as(_DP), _stream(stream)))
    return code, it, rr


def bw_lowest_modes(rve: Rve, k_list, nmodes: int, method: int = BW_SUBSPACE, block: int = 0, ncv: int = 0,
                    tol_eig: float = 0.0, tol_lin: float = 0.0, maxit_outer: int = 0, maxit_lin: int = 0,
                    warm_start: bool = True, modes=None, want_err: bool = True, tol_omega: float = 0.0,
                    kbatch: int = 0, net=None, kgroups: int = 0, stream=None):
    """omega (nk x nmodes, rad/s), error bounds, status and statistics.  net: a UNet for
    the learned preconditioner of the Lanczos inner solves (BW_LEARNED), else plain.
    kgroups > 1: the wave vectors in that many concurrent groups (Lanczos)."""
    k_arr, k_p = _darr(np.asarray(k_list).reshape(-1, 3))
    nk = int(k_arr.shape[0])
    om = np.zeros((nk, nmodes))
    er = np.zeros((nk, nmodes))
    opts = bw_eig_opts(method, block, ncv, maxit_outer, maxit_lin, int(bool(warm_start)), tol_eig, tol_lin,
                       tol_omega, kbatch, BW_LEARNED if net is not None else BW_PLAIN,
                       net.handle.value if net is not None else None, 0, int(kgroups))
    st = bw_stats()
    code = _check(lib().bw_lowest_modes(rve.handle, k_p, nk, int(nmodes), ctypes.byref(opts),
                                        om.ctypes.data_as(_DP), er.ctypes.data_as(_DP) if want_err else None,
                                        _dptr(modes) if modes is not None else None, ctypes.byref(st),
                                        _stream(stream)))
    return om, (er if want_err else None), code, st.as_dict()


def bw_lowest_modes_batched(rves, k_lists, nmodes: int, method: int = BW_SUBSPACE, block: int = 0, ncv: int = 0,
                            tol_eig: float = 0.0, tol_lin: float = 0.0, maxit_outer: int = 0, maxit_lin: int = 0,
                            warm_start: bool = True, tol_omega: float = 0.0, kbatch: int = 0, modes=None,
                            group_cells: bool = False, stream=None):
    """Several cells at once: lists of omega and error arrays, status, summed statistics.
    Every cell on a stream of its own; with group_cells (Lanczos), cells of one grid
    share every batched launch."""
    n = len(rves)
    ks = [np.ascontiguousarray(np.asarray(k).reshape(-1, 3), dtype=np.float64) for k in k_lists]
    oms = [np.zeros((k.shape[0], nmodes)) for k in ks]
    ers = [np.zeros((k.shape[0], nmodes)) for k in ks]
    h = (_P * n)(*[r.handle for r in rves])
    kp = (_DP * n)(*[k.ctypes.data_as(_DP) for k in ks])
    nk = (ctypes.c_int32 * n)(*[k.shape[0] for k in ks])
    op = (_DP * n)(*[o.ctypes.data_as(_DP) for o in oms])
    ep = (_DP * n)(*[e.ctypes.data_as(_DP) for e in ers])
    mp = (_P * n)(*[(_dptr(m) if m is not None else None) for m in modes]) if modes is not None else None
    opts = bw_eig_opts(method, block, ncv, maxit_outer, maxit_lin, int(bool(warm_start)), tol_eig, tol_lin,
                       tol_omega, kbatch, BW_PLAIN, None, int(bool(group_cells)))
    st = bw_stats()
    code = _check(lib().bw_lowest_modes_batched(h, n, kp, nk, int(nmodes), ctypes.byref(opts), op, ep, mp,
                                                ctypes.byref(st), _stream(stream)))
    return oms, ers, code, st.as_dict()


# ---------------------------------------------------------------------------
# dispersion post-processing
# ---------------------------------------------------------------------------
def bw_group_velocity(rve: Rve, k, direction, modes, omega, cluster_tol: float = 1e-6, stream=None) -> np.ndarray:
    """d omega / ds along `direction` for the modes at k (device tensor [nmodes][3][n0][n1][n2]
    as bw_lowest_modes writes it) with frequencies omega (rad/s, ascending); m/s."""
    nm = int(modes.shape[0])
    k_arr, k_p = _darr(np.asarray(k, dtype=np.float64).reshape(3))
    d_arr, d_p = _darr(np.asarray(direction, dtype=np.float64).reshape(3))
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(nm))
    out = np.zeros(nm)
    _check(lib().bw_group_velocity(rve.handle, k_p, d_p, nm, _dptr(modes), om.ctypes.data_as(_DP),
                                   float(cluster_tol), out.ctypes.data_as(_DP), _stream(stream)))
    return out


def bw_long_wave_speeds(rve: Rve, direction, h_frac: float = 0.02, tol_omega: float = 0.0, stream=None):
    """(speeds of the three acoustic branches along `direction` for k -> 0 (m/s, ascending), status)."""
    d_arr, d_p = _darr(np.asarray(direction, dtype=np.float64).reshape(3))
    out = np.zeros(3)
    code = _check(lib().bw_long_wave_speeds(rve.handle, d_p, float(h_frac), float(tol_omega),
                                            out.ctypes.data_as(_DP), _stream(stream)))
    return out, code


def bw_effective_stiffness(rve: Rve, rtol: float = 0.0, maxit: int = 0, stream=None):
    """(6 x 6 Voigt effective stiffness by static homogenization (Pa), PCG iterations of the
    six cell problems, status)."""
    C = np.zeros(36)
    it = np.zeros(6, dtype=np.int32)
    code = _check(lib().bw_effective_stiffness(rve.handle, float(rtol), int(maxit), C.ctypes.data_as(_DP),
                                               it.ctypes.data_as(_IP), _stream(stream)))
    return C.reshape(6, 6), it, code


def bw_mode_fields(rve: Rve, k, modes, u_out, eps_out=None, stream=None) -> np.ndarray:
    """Real-space displacement (and strain) fields of the modes at k; returns the phases."""
    nm = int(modes.shape[0])
    k_arr, k_p = _darr(np.asarray(k, dtype=np.float64).reshape(3))
    ph = np.zeros(nm)
    _check(lib().bw_mode_fields(rve.handle, k_p, nm, _dptr(modes), _dptr(u_out),
                                _dptr(eps_out) if eps_out is not None else None, ph.ctypes.data_as(_DP),
                                _stream(stream)))
    return ph


# ---------------------------------------------------------------------------
# learned preconditioner
# ---------------------------------------------------------------------------
def bw_unet_param_count() -> int:
    return int(lib().bw_unet_param_count())


class UNet:
    """Owning wrapper of a bw_unet handle (the network lives on the current device)."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check(lib().bw_unet_create(ctypes.byref(h), ctypes.c_uint64(int(seed))))
        self.handle = h
        self.nparam = bw_unet_param_count()

    def get_weights(self) -> np.ndarray:
        w = np.zeros(self.nparam, dtype=np.float32)
        _check(lib().bw_unet_get_weights(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), self.nparam))
        return w

    def set_weights(self, w) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        _check(lib().bw_unet_set_weights(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size))

    def close(self):
        if getattr(self, "handle", None):
            lib().bw_unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _grid(n):
    return (ctypes.c_int32 * 3)(*[int(v) for v in n])


def bw_unet_net_forward(net: UNet, n, x, y, stream=None) -> None:
    """y (nb, V, 16) = network(x (nb, V, 32)); float32 device tensors."""
    _check(lib().bw_unet_net_forward(net.handle, _grid(n), _dptr(x), _dptr(y), int(x.shape[0]), _stream(stream)))


def bw_unet_net_backward(net: UNet, n, x, dy, stream=None) -> np.ndarray:
    """Gradient of sum(dy * y(x)) with respect to the flat parameter vector."""
    g = np.zeros(net.nparam, dtype=np.float32)
    _check(lib().bw_unet_net_backward(net.handle, _grid(n), _dptr(x), _dptr(dy),
                                      g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(x.shape[0]),
                                      _stream(stream)))
    return g


def _klist(k, nrhs):
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    if k.shape[0] == 1 and nrhs > 1:
        k = np.repeat(k, nrhs, axis=0)
    if k.shape[0] != nrhs:
        raise ValueError("one wave vector, or one per right-hand side")
    return _darr(k)


def bw_unet_apply(net: UNet, rve: Rve, k, r, z, stream=None) -> None:
    nrhs = int(r.shape[0])
    k_arr, k_p = _klist(k, nrhs)
    _check(lib().bw_unet_apply(net.handle, rve.handle, k_p, _dptr(r), _dptr(z), nrhs, _stream(stream)))


def bw_unet_train_step(net: UNet, rve: Rve, k, r, x_star, lr: float, stream=None) -> float:
    nrhs = int(r.shape[0])
    k_arr, k_p = _klist(k, nrhs)
    loss = ctypes.c_double()
    _check(lib().bw_unet_train_step(net.handle, rve.handle, k_p, _dptr(r), _dptr(x_star), nrhs, float(lr),
                                    ctypes.byref(loss), _stream(stream)))
    return loss.value


def bw_unet_train_step_residual(net: UNet, rve: Rve, k, r, lr: float, stream=None) -> float:
    """One Adam step on mean ||K z - r||^2 / ||r||^2; returns the loss before the step."""
    nrhs = int(r.shape[0])
    k_arr, k_p = _klist(k, nrhs)
    loss = ctypes.c_double()
    _check(lib().bw_unet_train_step_residual(net.handle, rve.handle, k_p, _dptr(r), nrhs, float(lr),
                                             ctypes.byref(loss), _stream(stream)))
    return loss.value


def bw_pcg_solve_learned(rve: Rve, net, k, b, x, rtol: float, maxit: int = 0, stream=None):
    """Flexible PCG with the learned preconditioner (net None: plain P^);
    returns (status, iterations, true relative residuals, fallback counts)."""
    nrhs = int(b.shape[0])
    k_arr, k_p = _darr(k)
    it = np.zeros(nrhs, dtype=np.int32)
    rr = np.zeros(nrhs)
    fb = np.zeros(nrhs, dtype=np.int32)
    code = _check(lib().bw_pcg_solve_learned(rve.handle, net.handle if net is not None else None, k_p, _dptr(b),
                                             _dptr(x), nrhs, float(rtol), int(maxit), it.ctypes.data_as(_IP),
                                             rr.ctypes.data_as(_DP), fb.ctypes.data_as(_IP), _stream(stream)))
    return code, it, rr, fb
