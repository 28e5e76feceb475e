"""Thin ctypes binding of libnlinv.so (the C-ABI declared in include/nlinv.h).

Argument marshalling only: tensors are checked for device, dtype, shape and
contiguity and their data pointers are passed to the library, which enqueues
its HIP kernels on torch's current stream.  There is no fallback: if the
library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlinv.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nlinv.h")

OK, E_ARG, E_SIZE, E_WORKSPACE, E_HIP, E_STATE, E_NONFINITE, E_BUDGET = 0, -1, -2, -3, -4, -5, -6, -7
STATIC_WORKSPACE_BYTES = 128 << 20   # NLINV_STATIC_WORKSPACE_BYTES
F_EXACT_GRID, F_CHECK_FINITE = 2, 4
KT = {"none": 0, "toeplitz_rows": 1, "coil_cols": 2, "back_cols": 3, "cg_update": 4,
      "coil_rows": 5, "coilh_rows": 6, "grid": 7}


class NlinvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nlinv error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("G", ctypes.c_int32), ("J", ctypes.c_int32),
                ("K", ctypes.c_int32), ("S_r", ctypes.c_int32), ("U", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("newton", ctypes.c_int32), ("cg", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("alpha0", ctypes.c_double), ("alpha_q", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("sob_a", ctypes.c_double), ("sob_l", ctypes.c_double),
                ("col_tile", ctypes.c_int32), ("cg_passes", ctypes.c_int32), ("fft_split", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32


def load() -> ctypes.CDLL:
    """Load libnlinv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} not built: run `python -m paper_1701_08361_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "nlinv_params_default": [ctypes.POINTER(Params)],
        "nlinv_workspace_size": [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
        "nlinv_sizes": [ctypes.POINTER(Params), _P, _P, _P, _P, _P],
        "nlinv_plan_workspace_size": [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)],
        "nlinv_plan_create": [ctypes.POINTER(Params), _P, _P, ctypes.c_size_t, ctypes.POINTER(_P)],
        "nlinv_plan_create_static": [ctypes.POINTER(Params), _P, ctypes.POINTER(_P)],
        "nlinv_set_budget": [_I, ctypes.c_size_t],
        "nlinv_budget_used": [_I, ctypes.POINTER(ctypes.c_size_t)],
        "nlinv_plan_destroy": [_P],
        "nlinv_set_stream": [_P, _P],
        "nlinv_psf": [_P, _P, _I],
        "nlinv_psf_spokes": [_P, _P, _I, _I],
        "nlinv_psf_samples": [_P, _P, ctypes.c_int64, _I],
        "nlinv_grid": [_P, _P, _P, _P, _P],
        "nlinv_reconstruct": [_P, _P, _P, _P, _P, _I, _P, _P],
        "nlinv_reconstruct_frames": [_P, _I, _P, _P, _P, _P, _P, _P],
        "nlinv_set_batch": [_P, _I],
        "nlinv_get_batch": [_P],
        "nlinv_apply_F": [_P, _P, _P, _P],
        "nlinv_apply_DF": [_P, _P, _P, _P, _P],
        "nlinv_apply_DFH": [_P, _P, _P, _P, _P],
        "nlinv_apply_normal": [_P, _P, _P, ctypes.c_double, _P, _P],
        "nlinv_apply_WH": [_P, _P, _P],
        "nlinv_apply_normal2": [_P, _P, _P, _P, ctypes.c_double, _P, _P],
        "nlinv_apply_E": [_P, _P, _P, _P],
        "nlinv_apply_EH": [_P, _P, _P, _P],
        "nlinv_nudft": [_P, _P, _P, _P],
        "nlinv_newton_step": [_P, _P, _P, _P, ctypes.c_double, _I, _P],
        "nlinv_apply_normal_multi": [_I, _P, _P, _P, _P, _P, _P],
        "nlinv_reconstruct_multi": [_I, _P, _P, _P, _P, _P, _P, _P],
        "nlinv_set_coil_weights": [_P, _P],
        "nlinv_compress": [_P, _P, _I, _P, _P],
        "nlinv_compression_matrix": [_P, _P, _I, _P],
        "nlinv_coils": [_P, _P, _P, _P],
        "nlinv_sync": [_P],
        "nlinv_set_graphs": [_P, _I],
        "nlinv_timer_enable": [_P, _I],
        "nlinv_timer_read": [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32 if name == "nlinv_get_batch" else ctypes.c_int
    lib.nlinv_last_error.argtypes = [_P]
    lib.nlinv_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def header_symbols() -> list:
    """Names of the functions declared in include/nlinv.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|int32_t|const char\*)\s+(nlinv_\w+)\s*\(", text, re.M)))


def _check(rc: int, plan=None):
    if rc != OK:
        msg = load().nlinv_last_error(plan)
        raise NlinvError(rc, msg.decode() if msg else "")


def make_params(N: int, J: int, K: int, S_r: int = 0, U: int = 1, batch: int = 1, newton: int = 7,
                cg: int = 10, alpha0: float = 1.0, alpha_q: float = 0.5, alpha_min: float = 0.0,
                G: int = 0, sob_a: float = 880.0, sob_l: float = 16.0, flags: int = 0,
                col_tile: int = 0, cg_passes: int = 0, fft_split: int = 0) -> Params:
    p = Params()
    _check(load().nlinv_params_default(ctypes.byref(p)))
    p.N, p.G, p.J, p.K, p.S_r, p.U, p.batch = N, G, J, K, S_r, U, batch
    p.newton, p.cg, p.flags = newton, cg, flags
    p.alpha0, p.alpha_q, p.alpha_min, p.sob_a, p.sob_l = alpha0, alpha_q, alpha_min, sob_a, sob_l
    p.col_tile = col_tile
    p.cg_passes = cg_passes
    p.fft_split = fft_split
    return p


def workspace_size(p: Params) -> int:
    n = ctypes.c_size_t(0)
    _check(load().nlinv_workspace_size(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def set_budget(device: int, budget_bytes: int) -> None:
    """Cap the summed plan workspaces on HIP device `device` (0 = no cap);
    plan creation beyond it raises NlinvError with code E_BUDGET."""
    _check(load().nlinv_set_budget(int(device), int(budget_bytes)))


def budget_used(device: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load().nlinv_budget_used(int(device), ctypes.byref(n)))
    return n.value


def sizes(p: Params) -> dict:
    R, G, Gc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    S, X = ctypes.c_int64(), ctypes.c_int64()
    _check(load().nlinv_sizes(ctypes.byref(p), ctypes.byref(R), ctypes.byref(G), ctypes.byref(Gc),
                              ctypes.byref(S), ctypes.byref(X)))
    return {"R": R.value, "G": G.value, "Gc": Gc.value, "S": S.value, "X": X.value}


class Plan:
    """One NLINV plan: sizes, FP64 tables and a device workspace (a torch tensor)."""

    def __init__(self, N: int, J: int, K: int, device="cuda", static_workspace: bool = False, **kw):
        """static_workspace: take the library's static device array as the
        workspace (nlinv_plan_create_static: no device allocation; one such
        plan per GPU at a time) instead of a torch buffer."""
        import torch
        self.torch = torch
        self.lib = load()
        self.params = make_params(N, J, K, **kw)
        sz = sizes(self.params)
        self.N, self.J, self.K = N, J, K
        self.R, self.G, self.Gc, self.S, self.X = sz["R"], sz["G"], sz["Gc"], sz["S"], sz["X"]
        self.dtype = torch.complex64        # precision of the unknowns and linearisation points
        self.B = self.params.batch          # active batch (set_batch)
        self.Bmax = self.params.batch
        self.U = self.params.U
        self.S_r = self.S // K
        dev = torch.device(device)
        if dev.type != "cuda":
            raise ValueError("plans live on a GPU (device 'cuda' or 'cuda:k')")
        # the plan belongs to one device: resolve "cuda" to the current index
        self.device = torch.device("cuda", torch.cuda.current_device() if dev.index is None else dev.index)
        nbytes = workspace_size(self.params)
        self.ws_bytes = nbytes
        self.handle = None
        with torch.cuda.device(self.device):    # the library creates the plan on the current device
            self._stream = torch.cuda.current_stream(self.device).cuda_stream
            h = _P()
            if static_workspace:
                self._raw = self.ws = None
                _check(self.lib.nlinv_plan_create_static(ctypes.byref(self.params), _P(self._stream),
                                                         ctypes.byref(h)))
            else:
                raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
                off = (-raw.data_ptr()) % 256
                self._raw = raw
                self.ws = raw[off:off + nbytes]
                _check(self.lib.nlinv_plan_create(ctypes.byref(self.params), _P(self._stream),
                                                  _P(self.ws.data_ptr()), nbytes, ctypes.byref(h)))
        self.handle = h

    # -- helpers ---------------------------------------------------------
    def _stream_sync(self):
        cur = self.torch.cuda.current_device()
        if cur != self.device.index:
            raise RuntimeError(f"the plan lives on {self.device} but cuda:{cur} is current; "
                               f"call it inside torch.cuda.device({self.device.index})")
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            _check(self.lib.nlinv_set_stream(self.handle, _P(s)), self.handle)
            self._stream = s

    def _t(self, t, dtype, shape, name, allow_none=False):
        if t is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _ptr(self, t):
        return _P(t.data_ptr()) if t is not None else _P()

    def _turns(self, turns):
        if turns is None:
            return None
        if isinstance(turns, int):
            turns = [turns] * self.B
        if len(turns) != self.B:
            raise ValueError("one turn per batch item")
        return (ctypes.c_int32 * self.B)(*[int(t) for t in turns])

    def empty(self, *shape, dtype=None):
        return self.torch.empty(*shape, dtype=dtype or self.torch.complex64, device=self.device)

    # -- API -------------------------------------------------------------
    def psf(self, traj, turn: int, spokes: Optional[int] = None, samples: Optional[int] = None):
        """PSF kernel and gridding table of `turn` from traj [K][S_r][2]; with
        `spokes`, from its first `spokes` spokes only (nlinv_psf_spokes); with
        `samples`, from its first `samples` samples (nlinv_psf_samples)."""
        torch = self.torch
        self._t(traj, torch.float32, (self.K, self.S_r, 2), "traj")
        if spokes is not None and samples is not None:
            raise ValueError("give spokes or samples, not both")
        self._stream_sync()
        if samples is not None:
            _check(self.lib.nlinv_psf_samples(self.handle, self._ptr(traj), int(samples), int(turn)), self.handle)
        elif spokes is None:
            _check(self.lib.nlinv_psf(self.handle, self._ptr(traj), int(turn)), self.handle)
        else:
            _check(self.lib.nlinv_psf_spokes(self.handle, self._ptr(traj), int(spokes), int(turn)), self.handle)

    def grid(self, traj, y, turns: Optional[Sequence[int]] = None, z=None):
        torch = self.torch
        B, J, R = self.B, self.J, self.R
        self._t(traj, torch.float32, (B, self.K, self.S_r, 2), "traj")
        self._t(y, torch.complex64, (B, J, self.S), "y")
        if z is None:
            z = self.empty(B, J, R, R)
        self._t(z, torch.complex64, (B, J, R, R), "z")
        self._stream_sync()
        _check(self.lib.nlinv_grid(self.handle, self._ptr(traj), self._ptr(y), self._turns(turns),
                                   self._ptr(z)), self.handle)
        return z

    def reconstruct(self, z, turns, xprev=None, xhat=None, init: Optional[int] = None, img=None,
                    coils=None, want_img: bool = False, want_coils: bool = False):
        torch = self.torch
        B, J, R, X = self.B, self.J, self.R, self.X
        self._t(z, torch.complex64, (B, J, R, R), "z")
        self._t(xprev, torch.complex64, (B, X), "xprev", allow_none=True)
        if xhat is None:
            xhat = self.empty(B, X)
            if init is None:
                init = 2 if xprev is not None else 1
        elif init is None:
            init = 0
        self._t(xhat, torch.complex64, (B, X), "xhat")
        if want_img and img is None:
            img = self.empty(B, R, R, dtype=torch.float32)
        if want_coils and coils is None:
            coils = self.empty(B, J, R, R)
        self._t(img, torch.float32, (B, R, R), "img", allow_none=True)
        self._t(coils, torch.complex64, (B, J, R, R), "coils", allow_none=True)
        self._stream_sync()
        _check(self.lib.nlinv_reconstruct(self.handle, self._ptr(z), self._turns(turns), self._ptr(xprev),
                                          self._ptr(xhat), int(init), self._ptr(img), self._ptr(coils)),
               self.handle)
        return xhat, img, coils

    def set_batch(self, b: int):
        """Work on the first b items (1 <= b <= the plan's batch) from now on."""
        _check(self.lib.nlinv_set_batch(self.handle, int(b)), self.handle)
        self.B = int(self.lib.nlinv_get_batch(self.handle))

    def reconstruct_frames(self, z, turns, xprev=None, xhat=None, img=None, coils=None,
                           want_img: bool = False, want_coils: bool = False):
        """Consecutive frames z [count][J][R][R] of one series under the relaxed
        temporal coupling; xprev [X] is the frame before them (None: unit start)."""
        torch = self.torch
        J, R, X = self.J, self.R, self.X
        count = int(z.shape[0])
        self._t(z, torch.complex64, (count, J, R, R), "z")
        self._t(xprev, torch.complex64, (X,), "xprev", allow_none=True)
        xhat = self.empty(count, X) if xhat is None else xhat
        self._t(xhat, torch.complex64, (count, X), "xhat")
        if want_img and img is None:
            img = self.empty(count, R, R, dtype=torch.float32)
        if want_coils and coils is None:
            coils = self.empty(count, J, R, R)
        self._t(img, torch.float32, (count, R, R), "img", allow_none=True)
        self._t(coils, torch.complex64, (count, J, R, R), "coils", allow_none=True)
        if len(turns) != count:
            raise ValueError("one turn per frame")
        tt = (ctypes.c_int32 * count)(*[int(t) for t in turns])
        self._stream_sync()
        _check(self.lib.nlinv_reconstruct_frames(self.handle, count, self._ptr(z), tt, self._ptr(xprev),
                                                 self._ptr(xhat), self._ptr(img), self._ptr(coils)),
               self.handle)
        return xhat, img, coils

    def apply_F(self, traj, xhat, y=None):
        torch = self.torch
        self._t(traj, torch.float32, (self.B, self.K, self.S_r, 2), "traj")
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        y = self.empty(self.B, self.J, self.S) if y is None else y
        self._t(y, torch.complex64, (self.B, self.J, self.S), "y")
        self._stream_sync()
        _check(self.lib.nlinv_apply_F(self.handle, self._ptr(traj), self._ptr(xhat), self._ptr(y)), self.handle)
        return y

    def apply_DF(self, traj, xhat, dx, dy=None):
        torch = self.torch
        self._t(traj, torch.float32, (self.B, self.K, self.S_r, 2), "traj")
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._t(dx, torch.complex64, (self.B, self.X), "dx")
        dy = self.empty(self.B, self.J, self.S) if dy is None else dy
        self._t(dy, torch.complex64, (self.B, self.J, self.S), "dy")
        self._stream_sync()
        _check(self.lib.nlinv_apply_DF(self.handle, self._ptr(traj), self._ptr(xhat), self._ptr(dx),
                                       self._ptr(dy)), self.handle)
        return dy

    def apply_DFH(self, traj, xhat, dy, dx=None):
        torch = self.torch
        self._t(traj, torch.float32, (self.B, self.K, self.S_r, 2), "traj")
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._t(dy, torch.complex64, (self.B, self.J, self.S), "dy")
        dx = self.empty(self.B, self.X) if dx is None else dx
        self._t(dx, torch.complex64, (self.B, self.X), "dx")
        self._stream_sync()
        _check(self.lib.nlinv_apply_DFH(self.handle, self._ptr(traj), self._ptr(xhat), self._ptr(dy),
                                        self._ptr(dx)), self.handle)
        return dx

    def compression_matrix(self, y0, cc=None):
        """Compression transform [J][J_phys] from one calibration frame y0 [J_phys][S]."""
        torch = self.torch
        Jp = int(y0.shape[0])
        self._t(y0, torch.complex64, (Jp, self.S), "y0")
        cc = self.empty(self.J, Jp) if cc is None else cc
        self._t(cc, torch.complex64, (self.J, Jp), "cc")
        self._stream_sync()
        _check(self.lib.nlinv_compression_matrix(self.handle, self._ptr(y0), Jp, self._ptr(cc)), self.handle)
        return cc

    def compress(self, cc, yp, y=None):
        """Virtual channels y [B][J][S] = cc [J][J_phys] x yp [B][J_phys][S]."""
        torch = self.torch
        Jp = int(cc.shape[1])
        self._t(cc, torch.complex64, (self.J, Jp), "cc")
        self._t(yp, torch.complex64, (self.B, Jp, self.S), "yp")
        y = self.empty(self.B, self.J, self.S) if y is None else y
        self._t(y, torch.complex64, (self.B, self.J, self.S), "y")
        self._stream_sync()
        _check(self.lib.nlinv_compress(self.handle, self._ptr(cc), Jp, self._ptr(yp), self._ptr(y)), self.handle)
        return y

    def apply_WH(self, coils, xhat=None):
        """Adjoint of the coil synthesis: image block 0, coil blocks W^-H c_j."""
        torch = self.torch
        self._t(coils, torch.complex64, (self.B, self.J, self.R, self.R), "coils")
        xhat = self.empty(self.B, self.X) if xhat is None else xhat
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._stream_sync()
        _check(self.lib.nlinv_apply_WH(self.handle, self._ptr(coils), self._ptr(xhat)), self.handle)
        return xhat

    def apply_normal(self, turns, xhat, p, alpha: float = 0.0, q=None):
        torch = self.torch
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._t(p, torch.complex64, (self.B, self.X), "p")
        q = self.empty(self.B, self.X) if q is None else q
        self._t(q, torch.complex64, (self.B, self.X), "q")
        self._stream_sync()
        _check(self.lib.nlinv_apply_normal(self.handle, self._turns(turns), self._ptr(xhat), float(alpha),
                                           self._ptr(p), self._ptr(q)), self.handle)
        return q

    def apply_normal2(self, turns, xa, xb, p, alpha: float = 0.0, q=None):
        """q = DF_xa^H DF_xb p + alpha p through the PSF convolution; p, q complex128 [B][X]."""
        torch = self.torch
        self._t(xa, torch.complex64, (self.B, self.X), "xa")
        self._t(xb, torch.complex64, (self.B, self.X), "xb")
        self._t(p, torch.complex128, (self.B, self.X), "p")
        q = self.empty(self.B, self.X, dtype=torch.complex128) if q is None else q
        self._t(q, torch.complex128, (self.B, self.X), "q")
        self._stream_sync()
        _check(self.lib.nlinv_apply_normal2(self.handle, self._turns(turns), self._ptr(xa), self._ptr(xb),
                                            float(alpha), self._ptr(p), self._ptr(q)), self.handle)
        return q

    def apply_E(self, xhat, p, img=None):
        """Image-space derivative E_x p [B][J][R][R] (complex64) of p complex128 [B][X]."""
        torch = self.torch
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._t(p, torch.complex128, (self.B, self.X), "p")
        img = self.empty(self.B, self.J, self.R, self.R) if img is None else img
        self._t(img, torch.complex64, (self.B, self.J, self.R, self.R), "img")
        self._stream_sync()
        _check(self.lib.nlinv_apply_E(self.handle, self._ptr(xhat), self._ptr(p), self._ptr(img)), self.handle)
        return img

    def apply_EH(self, xhat, img, out=None):
        """E_x^H img, complex128 [B][X], of images [B][J][R][R] complex64."""
        torch = self.torch
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._t(img, torch.complex64, (self.B, self.J, self.R, self.R), "img")
        out = self.empty(self.B, self.X, dtype=torch.complex128) if out is None else out
        self._t(out, torch.complex128, (self.B, self.X), "out")
        self._stream_sync()
        _check(self.lib.nlinv_apply_EH(self.handle, self._ptr(xhat), self._ptr(img), self._ptr(out)), self.handle)
        return out

    def nudft(self, traj, img, y=None):
        """y = F img per channel [B][J][S] (exact non-uniform DFT)."""
        torch = self.torch
        self._t(traj, torch.float32, (self.B, self.K, self.S_r, 2), "traj")
        self._t(img, torch.complex64, (self.B, self.J, self.R, self.R), "img")
        y = self.empty(self.B, self.J, self.S) if y is None else y
        self._t(y, torch.complex64, (self.B, self.J, self.S), "y")
        self._stream_sync()
        _check(self.lib.nlinv_nudft(self.handle, self._ptr(traj), self._ptr(img), self._ptr(y)), self.handle)
        return y

    def newton_step(self, turns, z, xhat, alpha: float, cg: int, xprev=None):
        """One IRGNM update of xhat [B][X] complex64 in place (nlinv_newton_step)."""
        torch = self.torch
        self._t(z, torch.complex64, (self.B, self.J, self.R, self.R), "z")
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        self._t(xprev, torch.complex64, (self.B, self.X), "xprev", allow_none=True)
        self._stream_sync()
        _check(self.lib.nlinv_newton_step(self.handle, self._turns(turns), self._ptr(z), self._ptr(xprev),
                                          float(alpha), int(cg), self._ptr(xhat)), self.handle)
        return xhat

    def set_coil_weights(self, winv=None):
        """Use the table winv [Gc][Gc] of 1 / (G w') (stored as float32) as the
        Sobolev weight from now on (None: the plan's own).  The binding keeps
        the table alive while it is set."""
        torch = self.torch
        if winv is not None:
            winv = winv.to(device=self.device, dtype=torch.float32).contiguous()
        self._t(winv, torch.float32, (self.Gc, self.Gc), "winv", allow_none=True)
        _check(self.lib.nlinv_set_coil_weights(self.handle, self._ptr(winv)), self.handle)
        self._winv = winv

    def coils(self, xhat, coils=None, img=None, want_img: bool = True):
        torch = self.torch
        self._t(xhat, torch.complex64, (self.B, self.X), "xhat")
        coils = self.empty(self.B, self.J, self.R, self.R) if coils is None else coils
        if want_img and img is None:
            img = self.empty(self.B, self.R, self.R, dtype=torch.float32)
        self._stream_sync()
        _check(self.lib.nlinv_coils(self.handle, self._ptr(xhat), self._ptr(coils), self._ptr(img)), self.handle)
        return coils, img

    def set_graphs(self, enable: bool = True):
        _check(self.lib.nlinv_set_graphs(self.handle, 1 if enable else 0), self.handle)

    def timer_enable(self, kernel: str):
        _check(self.lib.nlinv_timer_enable(self.handle, KT[kernel]), self.handle)

    def timer_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.nlinv_timer_read(self.handle, ctypes.byref(ms), ctypes.byref(n)), self.handle)
        return ms.value, n.value

    def crop(self, img):
        """The N x N output image: the centre of an [..., R, R] array (rows and
        columns R/2 - floor(N/2) to R/2 + ceil(N/2) - 1; all of it when G = 2N)."""
        o = self.R // 2 - self.N // 2
        return img[..., o:o + self.N, o:o + self.N]

    def sync(self):
        _check(self.lib.nlinv_sync(self.handle), self.handle)

    def close(self):
        if getattr(self, "handle", None):
            with self.torch.cuda.device(self.device):
                self.lib.nlinv_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_multi(plans, zs, turns, xprevs=None, xhats=None, inits=None, imgs=None,
                      want_img: bool = False):
    """One frame on each plan as one launch (nlinv_reconstruct_multi): a HIP
    graph with one independent branch per plan, launched on the first plan's
    stream.  Per plan i: zs[i] [B][J][R][R], turns[i] (B turns), xprevs[i]
    [B][X] or None, xhats[i] [B][X] (allocated if None), inits[i] as in
    Plan.reconstruct, imgs[i] [B][R][R] float32 or None.  Returns (xhats, imgs)."""
    import torch
    n = len(plans)
    xprevs = [None] * n if xprevs is None else list(xprevs)
    xhats = [None] * n if xhats is None else list(xhats)
    inits = [None] * n if inits is None else list(inits)
    imgs = [None] * n if imgs is None else list(imgs)
    if not (len(zs) == len(turns) == len(xprevs) == len(xhats) == len(inits) == len(imgs) == n):
        raise ValueError("one set of arguments per plan")
    for i, pl in enumerate(plans):
        pl._t(zs[i], torch.complex64, (pl.B, pl.J, pl.R, pl.R), "z")
        pl._t(xprevs[i], torch.complex64, (pl.B, pl.X), "xprev", allow_none=True)
        if xhats[i] is None:
            xhats[i] = pl.empty(pl.B, pl.X)
            if inits[i] is None:
                inits[i] = 2 if xprevs[i] is not None else 1
        elif inits[i] is None:
            inits[i] = 0
        pl._t(xhats[i], torch.complex64, (pl.B, pl.X), "xhat")
        if want_img and imgs[i] is None:
            imgs[i] = pl.empty(pl.B, pl.R, pl.R, dtype=torch.float32)
        pl._t(imgs[i], torch.float32, (pl.B, pl.R, pl.R), "img", allow_none=True)
    plans[0]._stream_sync()
    P = ctypes.c_void_p
    handles = (P * n)(*[pl.handle for pl in plans])
    tl = [plans[i]._turns(turns[i]) for i in range(n)]
    tp = (P * n)(*[ctypes.cast(t, P) for t in tl])
    zp = (P * n)(*[z.data_ptr() for z in zs])
    pp = (P * n)(*[(x.data_ptr() if x is not None else None) for x in xprevs])
    xp = (P * n)(*[x.data_ptr() for x in xhats])
    ip = (ctypes.c_int32 * n)(*[int(v) for v in inits])
    gp = (P * n)(*[(g.data_ptr() if g is not None else None) for g in imgs])
    rc = load().nlinv_reconstruct_multi(n, handles, zp, tp, pp, xp, ip, gp)
    if rc != OK:
        msgs = [load().nlinv_last_error(h) for h in [pl.handle for pl in plans] + [None]]
        msg = next((m.decode() for m in msgs if m), "")
        raise NlinvError(rc, msg)
    return xhats, imgs


def apply_normal_multi(plans, turns, xhats, alphas, ps, qs=None):
    """The CG operator of several plans of different grid sides (256, 320,
    384) with one ragged Toeplitz launch (nlinv_apply_normal_multi); equals
    Plan.apply_normal per plan.  Runs on the first plan's stream."""
    import torch
    n = len(plans)
    if not (len(turns) == len(xhats) == len(alphas) == len(ps) == n):
        raise ValueError("one turn list, point, alpha and direction per plan")
    qs = [pl.empty(pl.B, pl.X) for pl in plans] if qs is None else qs
    for pl, x, p, q in zip(plans, xhats, ps, qs):
        for t, name in ((x, "xhat"), (p, "p"), (q, "q")):
            pl._t(t, torch.complex64, (pl.B, pl.X), name)
    plans[0]._stream_sync()
    P = ctypes.c_void_p
    handles = (P * n)(*[pl.handle for pl in plans])
    tl = [plans[i]._turns(turns[i]) for i in range(n)]
    tp = (P * n)(*[ctypes.cast(t, P) for t in tl])
    xp = (P * n)(*[x.data_ptr() for x in xhats])
    pp = (P * n)(*[p.data_ptr() for p in ps])
    qp = (P * n)(*[q.data_ptr() for q in qs])
    ap = (ctypes.c_double * n)(*[float(a) for a in alphas])
    rc = load().nlinv_apply_normal_multi(n, handles, tp, xp, ap, pp, qp)
    if rc != OK:
        msgs = [load().nlinv_last_error(h) for h in [pl.handle for pl in plans] + [None]]
        msg = next((m.decode() for m in msgs if m), "")
        raise NlinvError(rc, msg)
    return qs
