"""ctypes binding of libqc (include/qc.h): argument marshalling only.

Every step of the solve runs in the HIP kernels of libqc.so; this module
only checks tensor dtypes/devices/contiguity, fills the C structs with
device pointers and calls the library.  It raises if the library is not
built: there is no other code path.

Arrays are torch tensors on the HIP device (the layouts are those of
include/qc.h).  Visibility sets and chain terms are the plain containers
of ``synth.problem`` (Vis, Term) holding such tensors.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqc.so")

QC_OK, QC_E_ARG, QC_E_RANGE, QC_E_NONFINITE, QC_E_DEVICE, QC_E_NOMEM, QC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "QC_OK", -1: "QC_E_ARG", -2: "QC_E_RANGE", -3: "QC_E_NONFINITE", -4: "QC_E_DEVICE",
                -5: "QC_E_NOMEM", -6: "QC_E_UNSUPPORTED"}
TERM_TYPES = {"diag": 0, "c2x2": 1, "delay": 2, "phase": 3, "amplitude": 4, "delay_offset": 5, "pointing": 6}
PRECISIONS = {"fp64": 0, "mixed": 1}
DAMPINGS = {"full": 0, "half": 1, "alternate": 2, "auto": 3, "lm": 4}

EXPORTS = ("qc_ctx_create", "qc_ctx_destroy", "qc_ctx_sync", "qc_last_error", "qc_last_kernel_ms", "qc_ctx_set_tile",
           "qc_ctx_set_split", "qc_ctx_last_split",
           "qc_solve_interval", "qc_solve_interval_static", "qc_solve_chain", "qc_delay_init", "qc_apply_gains", "qc_residual",
           "qc_batch_create", "qc_batch_tune", "qc_batch_run", "qc_batch_last_ms", "qc_batch_schedule",
           "qc_batch_destroy", "qc_solve_batch", "qc_ws_features", "qc_mlp_forward", "qc_mlp_backward",
           "qc_adam_step", "qc_mse_grad", "qc_ws_gains", "qc_ws_labels", "qc_mad_flag", "qc_predict_dft", "qc_robust_weights",
           "qc_corrected_weights", "qc_solve_chain_robust", "qc_interp_term", "qc_solve_interval_sky",
           "qc_residual_sky", "qc_corrupt_sky", "qc_batch_n_intervals", "qc_batch_ws_features", "qc_batch_ws_gains")
MAD_MODES = {"global": 0, "baseline": 1}
BATCH_BUCKETS = 6


class QcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class QcVis(C.Structure):
    _fields_ = [("n_row", C.c_int64), ("n_chan", C.c_int32), ("n_dir", C.c_int32), ("n_ant", C.c_int32),
                ("n_time", C.c_int32), ("n_wcorr", C.c_int32), ("dtype", C.c_int32),
                ("data", C.c_void_p), ("model", C.c_void_p), ("weight", C.c_void_p), ("flag", C.c_void_p),
                ("ant1", C.c_void_p), ("ant2", C.c_void_p), ("row_time", C.c_void_p), ("chan_freq", C.c_void_p)]


class QcTerm(C.Structure):
    _fields_ = [("type", C.c_int32), ("direction_dependent", C.c_int32), ("n_gt", C.c_int32),
                ("n_gf", C.c_int32), ("n_gdir", C.c_int32),
                ("t_map", C.c_void_p), ("f_map", C.c_void_p), ("d_map", C.c_void_p),
                ("gains", C.c_void_p), ("params", C.c_void_p), ("gain_flags", C.c_void_p),
                ("dir_lm", C.c_void_p), ("beam_fwhm", C.c_double), ("beam_freq", C.c_double)]


class QcSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("prec", C.c_int32), ("damping", C.c_int32),
                ("stream", C.c_void_p), ("chisq_ref", C.c_void_p)]


class QcSolveStats(C.Structure):
    _fields_ = [("iters", C.c_void_p), ("converged", C.c_void_p), ("chisq_first", C.c_void_p),
                ("chisq_last", C.c_void_p), ("restarted", C.c_void_p)]


class QcProblem(C.Structure):
    _fields_ = [("vis", QcVis), ("term", QcTerm), ("stats", QcSolveStats), ("chisq_ref", C.c_void_p)]


class QcSky(C.Structure):
    _fields_ = [("n_comp", C.c_int64), ("lm", C.c_void_p), ("stokes", C.c_void_p), ("spi", C.c_void_p),
                ("ref_freq", C.c_void_p), ("dir", C.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libqc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libqc.so not built at {path}; run python -m paper_2412_10072_amd.build")
    lib = C.CDLL(path)
    lib.qc_ctx_create.argtypes = [C.c_int32, C.POINTER(C.c_void_p)]
    lib.qc_ctx_destroy.argtypes = [C.c_void_p]
    lib.qc_ctx_sync.argtypes = [C.c_void_p]
    lib.qc_last_error.argtypes = [C.c_void_p]
    lib.qc_last_error.restype = C.c_char_p
    lib.qc_last_kernel_ms.argtypes = [C.c_void_p]
    lib.qc_last_kernel_ms.restype = C.c_double
    lib.qc_solve_interval.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32, C.c_int32,
                                      C.POINTER(QcSolveOpts), C.POINTER(QcSolveStats)]
    lib.qc_solve_interval_static.argtypes = lib.qc_solve_interval.argtypes
    lib.qc_solve_interval_sky.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcSky), C.c_void_p,
                                          C.POINTER(QcTerm), C.c_int32, C.c_int32, C.POINTER(QcSolveOpts),
                                          C.POINTER(QcSolveStats)]
    lib.qc_residual_sky.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcSky), C.c_void_p, C.POINTER(QcTerm),
                                    C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.qc_corrupt_sky.argtypes = lib.qc_residual_sky.argtypes
    lib.qc_ctx_set_tile.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    lib.qc_ctx_set_split.argtypes = [C.c_void_p, C.c_int32]
    lib.qc_ctx_last_split.argtypes = [C.c_void_p]
    lib.qc_ctx_last_split.restype = C.c_int32
    lib.qc_solve_chain.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32, C.c_int32,
                                   C.POINTER(QcSolveOpts), C.c_void_p]
    lib.qc_delay_init.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32, C.c_void_p]
    lib.qc_apply_gains.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
    lib.qc_residual.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32,
                                C.c_void_p, C.c_void_p, C.c_void_p]
    lib.qc_mad_flag.argtypes = [C.c_void_p, C.POINTER(QcVis), C.c_void_p, C.c_int32, C.c_double, C.c_void_p,
                                C.c_void_p, C.POINTER(C.c_int64), C.c_void_p]
    lib.qc_interp_term.argtypes = [C.c_void_p, C.POINTER(QcTerm), C.c_void_p, C.c_void_p, C.POINTER(QcTerm),
                                   C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.qc_solve_chain_robust.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32, C.c_int32,
                                          C.POINTER(QcSolveOpts), C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.qc_robust_weights.argtypes = [C.c_void_p, C.POINTER(QcVis), C.c_void_p, C.c_double, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
    lib.qc_corrected_weights.argtypes = [C.c_void_p, C.POINTER(QcVis), C.POINTER(QcTerm), C.c_int32, C.c_void_p,
                                         C.c_void_p]
    lib.qc_predict_dft.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.POINTER(QcSky),
                                   C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
    lib.qc_batch_create.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(QcSolveOpts), C.POINTER(C.c_void_p)]
    lib.qc_batch_tune.argtypes = [C.c_void_p, C.c_int32]
    lib.qc_batch_run.argtypes = [C.c_void_p, C.c_void_p]
    lib.qc_batch_last_ms.argtypes = [C.c_void_p]
    lib.qc_batch_last_ms.restype = C.c_double
    lib.qc_batch_schedule.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]
    lib.qc_batch_destroy.argtypes = [C.c_void_p]
    lib.qc_solve_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(QcSolveOpts)]
    vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
    lib.qc_ws_features.argtypes = [vp, C.POINTER(QcVis), C.POINTER(QcTerm), vp, vp, i32, vp]
    lib.qc_mlp_forward.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp, vp]
    lib.qc_mlp_backward.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp]
    lib.qc_adam_step.argtypes = [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32, i32, vp]
    lib.qc_mse_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.qc_ws_gains.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.qc_ws_labels.argtypes = [vp, vp, i32, i32, i32, vp, vp]
    lib.qc_batch_n_intervals.argtypes = [vp]
    lib.qc_batch_ws_features.argtypes = [vp, vp, i32, vp, i32, vp]
    lib.qc_batch_ws_gains.argtypes = [vp, vp, i32, vp]
    for name in EXPORTS:
        if name not in ("qc_last_error", "qc_last_kernel_ms", "qc_batch_last_ms", "qc_ctx_last_split"):
            getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(t: Optional[torch.Tensor], dtype=None, name="array") -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, got {type(t)}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the HIP device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def to_device(x, device, dtype=None) -> torch.Tensor:
    t = torch.as_tensor(np.ascontiguousarray(x) if isinstance(x, np.ndarray) else x)
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device).contiguous()


def device_vis(vis, device="cuda"):
    """Copy of a visibility container with every array on `device`."""
    from synth.problem import Vis
    return Vis(data=to_device(vis.data, device), model=to_device(vis.model, device),
               weight=to_device(vis.weight, device), flag=to_device(vis.flag, device, torch.uint8),
               ant1=to_device(vis.ant1, device, torch.int32), ant2=to_device(vis.ant2, device, torch.int32),
               row_time=to_device(vis.row_time, device, torch.int32),
               chan_freq=to_device(vis.chan_freq, device, torch.float64), n_ant=int(vis.n_ant),
               n_time=int(vis.n_time))


def device_term(term, device="cuda"):
    """Copy of a chain term with every array on `device` (gains complex128)."""
    t = term.copy()
    t.t_map = to_device(term.t_map, device, torch.int32)
    t.f_map = to_device(term.f_map, device, torch.int32)
    t.d_map = to_device(term.d_map, device, torch.int32)
    t.gains = to_device(term.gains, device, torch.complex128) if term.gains is not None else None
    t.params = to_device(term.params, device, torch.float64) if term.params is not None else None
    if getattr(term, "dir_lm", None) is not None:
        t.dir_lm = to_device(term.dir_lm, device, torch.float64)
    if term.gain_flags is not None:
        gf = term.gain_flags
    else:
        g = term.gains if term.gains is not None else term.params
        gf = np.zeros(tuple(g.shape[:4]), np.int8)
    t.gain_flags = to_device(gf, device, torch.int8)
    return t


def host_term(term):
    """Copy of a chain term with every array as numpy (for comparisons)."""
    t = term.copy()
    for name in ("t_map", "f_map", "d_map", "gains", "params", "gain_flags", "dir_lm"):
        v = getattr(term, name)
        if isinstance(v, torch.Tensor):
            setattr(t, name, v.detach().cpu().numpy())
    return t


def _c_vis(vis, n_dir: Optional[int] = None) -> QcVis:
    """vis.model may be None when n_dir is given (a model predicted from a sky)."""
    data = vis.data
    if data.dtype == torch.complex64:
        dtype, wdt = 0, torch.float32
    elif data.dtype == torch.complex128:
        dtype, wdt = 1, torch.float64
    else:
        raise TypeError(f"data must be complex64 or complex128, got {data.dtype}")
    n_row, n_chan = int(data.shape[0]), int(data.shape[1])
    if tuple(data.shape) != (n_row, n_chan, 4):
        raise ValueError(f"data must be [n_row][n_chan][4], got {tuple(data.shape)}")
    if vis.model is None:
        if n_dir is None:
            raise ValueError("vis.model is None: give the number of model directions")
    elif vis.model.dim() != 4 or tuple(vis.model.shape[:2]) != (n_row, n_chan) or vis.model.shape[3] != 4:
        raise ValueError(f"model must be [n_row][n_chan][n_dir][4], got {tuple(vis.model.shape)}")
    if vis.weight.dim() != 3 or tuple(vis.weight.shape[:2]) != (n_row, n_chan):
        raise ValueError(f"weight must be [n_row][n_chan][n_wcorr], got {tuple(vis.weight.shape)}")
    if tuple(vis.flag.shape) != (n_row, n_chan):
        raise ValueError("flag must be [n_row][n_chan]")
    for name in ("ant1", "ant2", "row_time"):
        if tuple(getattr(vis, name).shape) != (n_row,):
            raise ValueError(f"{name} must be [n_row]")
    if tuple(vis.chan_freq.shape) != (n_chan,):
        raise ValueError("chan_freq must be [n_chan]")
    nd = int(n_dir) if vis.model is None else int(vis.model.shape[2])
    if n_dir is not None and int(n_dir) != nd:
        raise ValueError(f"n_dir={n_dir} differs from the model's {nd} directions")
    return QcVis(n_row=n_row, n_chan=n_chan, n_dir=nd, n_ant=int(vis.n_ant),
                 n_time=int(vis.n_time), n_wcorr=int(vis.weight.shape[2]), dtype=dtype,
                 data=_ptr(data, name="data"), model=_ptr(vis.model, data.dtype, "model"),
                 weight=_ptr(vis.weight, wdt, "weight"), flag=_ptr(vis.flag, torch.uint8, "flag"),
                 ant1=_ptr(vis.ant1, torch.int32, "ant1"), ant2=_ptr(vis.ant2, torch.int32, "ant2"),
                 row_time=_ptr(vis.row_time, torch.int32, "row_time"),
                 chan_freq=_ptr(vis.chan_freq, torch.float64, "chan_freq"))


def _c_chain(chain: Sequence) -> C.Array:
    arr = (QcTerm * len(chain))()
    for j, t in enumerate(chain):
        if t.kind not in TERM_TYPES:
            raise ValueError(f"term {j}: unknown kind {t.kind!r}")
        c = arr[j]
        c.type = TERM_TYPES[t.kind]
        c.direction_dependent = 1 if t.direction_dependent else 0
        c.n_gt, c.n_gf, c.n_gdir = int(t.n_gt), int(t.n_gf), int(t.n_gdir)
        c.t_map = _ptr(t.t_map, torch.int32, "t_map")
        c.f_map = _ptr(t.f_map, torch.int32, "f_map")
        c.d_map = _ptr(t.d_map, torch.int32, "d_map")
        c.gains = _ptr(t.gains, torch.complex128, "gains") if t.gains is not None else None
        c.params = _ptr(t.params, torch.float64, "params") if t.params is not None else None
        c.gain_flags = _ptr(t.gain_flags, torch.int8, "gain_flags") if t.gain_flags is not None else None
        if t.kind == "pointing":
            if t.dir_lm is None or t.beam is None:
                raise ValueError(f"term {j}: a pointing term needs dir_lm and beam")
            c.dir_lm = _ptr(t.dir_lm, torch.float64, "dir_lm")
            c.beam_fwhm, c.beam_freq = float(t.beam[0]), float(t.beam[1])
    return arr


@dataclass
class Sky:
    """Point components on the device: lm [n_comp][2], stokes [n_comp][4] (I, Q, U,
    V), spi [n_comp], ref_freq [n_comp] float64, comp_dir [n_comp] int32, with the
    rows' baseline coordinates uvw [n_row][3] float64 and the number of model
    directions n_dir."""
    lm: torch.Tensor
    stokes: torch.Tensor
    spi: torch.Tensor
    ref_freq: torch.Tensor
    comp_dir: torch.Tensor
    uvw: torch.Tensor
    n_dir: int

    def c(self) -> "QcSky":
        n = int(self.lm.shape[0])
        if tuple(self.lm.shape) != (n, 2) or tuple(self.stokes.shape) != (n, 4) or self.spi.numel() != n \
                or self.ref_freq.numel() != n or self.comp_dir.numel() != n or self.uvw.dim() != 2 \
                or self.uvw.shape[1] != 3:
            raise ValueError("inconsistent component or uvw shapes")
        return QcSky(n_comp=n, lm=_ptr(self.lm, torch.float64, "lm"), stokes=_ptr(self.stokes, torch.float64, "stokes"),
                     spi=_ptr(self.spi, torch.float64, "spi"), ref_freq=_ptr(self.ref_freq, torch.float64, "ref_freq"),
                     dir=_ptr(self.comp_dir, torch.int32, "comp_dir"))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class _Shape1:
    n_gt = n_gf = 1


def _stats_for(term, dev):
    shape = (int(term.n_gt), int(term.n_gf))
    return dict(iters=torch.zeros(shape, dtype=torch.int32, device=dev),
                converged=torch.zeros(shape, dtype=torch.uint8, device=dev),
                chisq_first=torch.zeros(shape, dtype=torch.float64, device=dev),
                chisq_last=torch.zeros(shape, dtype=torch.float64, device=dev),
                restarted=torch.zeros(shape, dtype=torch.uint8, device=dev))


def _c_stats(st) -> QcSolveStats:
    return QcSolveStats(iters=_ptr(st["iters"], torch.int32, "iters"),
                        converged=_ptr(st["converged"], torch.uint8, "converged"),
                        chisq_first=_ptr(st["chisq_first"], torch.float64, "chisq_first"),
                        chisq_last=_ptr(st["chisq_last"], torch.float64, "chisq_last"),
                        restarted=_ptr(st.get("restarted"), torch.uint8, "restarted"))


def _f32(t, name):
    return _ptr(t, torch.float32, name)


class Context:
    """A libqc context on one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        st = self.lib.qc_ctx_create(device, C.byref(h))
        if st != QC_OK:
            raise QcError(st, f"qc_ctx_create({device}) failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.qc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != QC_OK:
            raise QcError(st, self.lib.qc_last_error(self.h).decode())

    def sync(self):
        self._check(self.lib.qc_ctx_sync(self.h))

    def set_tile(self, waves: int = 0, rows_per_step: int = 0):
        """qc_ctx_set_tile: launch shape of the per-interval solve (0 = default)."""
        self._check(self.lib.qc_ctx_set_tile(self.h, int(waves), int(rows_per_step)))

    def set_split(self, parts: int = 0):
        """qc_ctx_set_split: 0 automatic, 1 never split, > 1 parts per interval."""
        self._check(self.lib.qc_ctx_set_split(self.h, int(parts)))

    def last_split_parts(self) -> int:
        return int(self.lib.qc_ctx_last_split(self.h))

    def last_kernel_ms(self) -> float:
        return float(self.lib.qc_last_kernel_ms(self.h))

    def solve(self, vis, chain, active: int = 0, tol: float = 1e-6, max_iter: int = 100,
              prec: str = "mixed", damping: str = "auto", stream=None, stats: Optional[dict] = None,
              chisq_ref: Optional[torch.Tensor] = None, static: bool = False):
        """qc_solve_interval: solve chain[active] in place; returns the per-interval stats tensors.
        chisq_ref (per interval, float64): restart an interval from unit gains when chi^2 at its
        starting gains exceeds the entry (warm-start fallback).  static: call
        qc_solve_interval_static (no device allocation inside the library; pass `stats`
        to allocate nothing here either)."""
        dev = vis.data.device
        # an out-of-range `active` is passed on: the library rejects it with QC_E_ARG
        term = chain[active] if 0 <= active < len(chain) else None
        if stats is None:
            stats = _stats_for(term, dev) if term is not None else _stats_for(_Shape1(), dev)
        cv = _c_vis(vis)
        cc = _c_chain(chain)
        opts = QcSolveOpts(tol=float(tol), max_iter=int(max_iter), prec=PRECISIONS[prec],
                           damping=DAMPINGS[damping], stream=_stream_ptr(stream),
                           chisq_ref=_ptr(chisq_ref, torch.float64, "chisq_ref"))
        cs = _c_stats(stats)
        fn = self.lib.qc_solve_interval_static if static else self.lib.qc_solve_interval
        self._check(fn(self.h, C.byref(cv), cc, len(chain), int(active), C.byref(opts), C.byref(cs)))
        return stats

    def solve_sky(self, vis, sky: "Sky", chain, active: int = 0, tol: float = 1e-6, max_iter: int = 100,
                  prec: str = "mixed", damping: str = "auto", stream=None, stats: Optional[dict] = None):
        """qc_solve_interval_sky: as solve, with the model predicted from `sky` inside the
        solver's passes (vis.model is not read and may be None)."""
        dev = vis.data.device
        term = chain[active] if 0 <= active < len(chain) else None
        if stats is None:
            stats = _stats_for(term, dev) if term is not None else _stats_for(_Shape1(), dev)
        cv = _c_vis(vis, sky.n_dir)
        cc = _c_chain(chain)
        opts = QcSolveOpts(tol=float(tol), max_iter=int(max_iter), prec=PRECISIONS[prec],
                           damping=DAMPINGS[damping], stream=_stream_ptr(stream))
        cs = _c_stats(stats)
        csky = sky.c()
        self._check(self.lib.qc_solve_interval_sky(self.h, C.byref(cv), C.byref(csky),
                                                   C.c_void_p(_ptr(sky.uvw, torch.float64, "uvw")), cc, len(chain),
                                                   int(active), C.byref(opts), C.byref(cs)))
        return stats

    def residual_sky(self, vis, sky: "Sky", chain, dir_mask=None, out=None, stream=None, corrupt: bool = False):
        """qc_residual_sky (or qc_corrupt_sky): the residual (corrupted model) with the model
        predicted from `sky`."""
        if out is None:
            out = torch.empty_like(vis.data)
        if tuple(out.shape) != tuple(vis.data.shape) or out.dtype != vis.data.dtype:
            raise ValueError("out must be shaped and typed like vis.data")
        mp = None
        if dir_mask is not None:
            keep = np.ascontiguousarray(np.asarray(dir_mask, dtype=np.uint8))
            if keep.size != sky.n_dir:
                raise ValueError("dir_mask needs one entry per direction")
            mp = keep.ctypes.data_as(C.c_void_p)
        cv = _c_vis(vis, sky.n_dir)
        cc = _c_chain(chain)
        csky = sky.c()
        fn = self.lib.qc_corrupt_sky if corrupt else self.lib.qc_residual_sky
        self._check(fn(self.h, C.byref(cv), C.byref(csky), C.c_void_p(_ptr(sky.uvw, torch.float64, "uvw")), cc,
                       len(chain), mp, C.c_void_p(out.data_ptr()), C.c_void_p(_stream_ptr(stream))))
        return out

    def solve_chain(self, vis, chain, n_epoch: int = 1, tol: float = 1e-6, max_iter: int = 100,
                    prec: str = "mixed", damping: str = "auto", stream=None):
        """qc_solve_chain: every term solved in turn, n_epoch passes; returns [epoch][term] stats."""
        dev = vis.data.device
        stats, cstats = [], (QcSolveStats * max(1, n_epoch * len(chain)))()
        for e in range(n_epoch):
            row = []
            for n, term in enumerate(chain):
                st = _stats_for(term, dev)
                cstats[e * len(chain) + n] = _c_stats(st)
                row.append(st)
            stats.append(row)
        cv = _c_vis(vis)
        cc = _c_chain(chain)
        opts = QcSolveOpts(tol=float(tol), max_iter=int(max_iter), prec=PRECISIONS[prec],
                           damping=DAMPINGS[damping], stream=_stream_ptr(stream))
        self._check(self.lib.qc_solve_chain(self.h, C.byref(cv), cc, len(chain), int(n_epoch), C.byref(opts),
                                            C.cast(cstats, C.c_void_p)))
        return stats

    def solve_chain_robust(self, vis, chain, n_epoch: int = 2, nu: float = 2.0, tol: float = 1e-6,
                           max_iter: int = 100, prec: str = "mixed", damping: str = "auto", resid_work=None,
                           weight_work=None, stream=None):
        """qc_solve_chain_robust: qc_solve_chain with robust reweighting between
        epochs; returns ([epoch][term] stats, the weights of the last epoch)."""
        dev = vis.data.device
        stats, cstats = [], (QcSolveStats * max(1, n_epoch * len(chain)))()
        for e in range(n_epoch):
            row = []
            for n, term in enumerate(chain):
                st = _stats_for(term, dev)
                cstats[e * len(chain) + n] = _c_stats(st)
                row.append(st)
            stats.append(row)
        if resid_work is None:
            resid_work = torch.empty_like(vis.data)
        if weight_work is None:
            weight_work = torch.empty_like(vis.weight)
        if tuple(resid_work.shape) != tuple(vis.data.shape) or resid_work.dtype != vis.data.dtype \
                or tuple(weight_work.shape) != tuple(vis.weight.shape) or weight_work.dtype != vis.weight.dtype:
            raise ValueError("work arrays must be shaped and typed like vis.data and vis.weight")
        cv = _c_vis(vis)
        cc = _c_chain(chain)
        opts = QcSolveOpts(tol=float(tol), max_iter=int(max_iter), prec=PRECISIONS[prec],
                           damping=DAMPINGS[damping], stream=_stream_ptr(stream))
        self._check(self.lib.qc_solve_chain_robust(self.h, C.byref(cv), cc, len(chain), int(n_epoch),
                                                   C.byref(opts), float(nu),
                                                   C.c_void_p(_ptr(resid_work, vis.data.dtype, "resid_work")),
                                                   C.c_void_p(_ptr(weight_work, vis.weight.dtype, "weight_work")),
                                                   C.cast(cstats, C.c_void_p)))
        return stats, (weight_work if n_epoch > 1 else vis.weight)

    def delay_init(self, vis, term, ref_ant: int = 0, stream=None):
        """qc_delay_init: Fourier-peak delay estimate written into term.params."""
        cv = _c_vis(vis)
        cc = _c_chain([term])
        self._check(self.lib.qc_delay_init(self.h, C.byref(cv), cc, int(ref_ant), C.c_void_p(_stream_ptr(stream))))
        return term

    # ---- learned warm start ----------------------------------------------

    def ws_features(self, vis, layout, feat: Optional[torch.Tensor] = None,
                    chisq_unit: Optional[torch.Tensor] = None, ref_ant: int = -1, stream=None):
        """qc_ws_features: per-interval features [n_int][n_ant*8] (float32), referenced to
        ref_ant when >= 0, and, if given, chi^2 at unit gains per interval (float64)."""
        n_int = int(layout.n_gt) * int(layout.n_gf)
        if feat is None:
            feat = torch.empty(n_int, int(vis.n_ant) * 8, dtype=torch.float32, device=vis.data.device)
        if tuple(feat.shape) != (n_int, int(vis.n_ant) * 8):
            raise ValueError("feat must be [n_int][n_ant*8]")
        cv = _c_vis(vis)
        cc = _c_chain([layout])
        self._check(self.lib.qc_ws_features(self.h, C.byref(cv), cc, C.c_void_p(_f32(feat, "feat")),
                                            C.c_void_p(_ptr(chisq_unit, torch.float64, "chisq_unit")),
                                            int(ref_ant), C.c_void_p(_stream_ptr(stream))))
        return feat

    def mlp_forward(self, params, x, n_hid: int, n_out: int, y=None, pre=None, stream=None):
        B, n_in = int(x.shape[0]), int(x.shape[1])
        dev = x.device
        y = torch.empty(B, n_out, dtype=torch.float32, device=dev) if y is None else y
        pre = torch.empty(B, n_hid, dtype=torch.float32, device=dev) if pre is None else pre
        self._check(self.lib.qc_mlp_forward(self.h, _f32(params, "params"), _f32(x, "x"), B, n_in, n_hid, n_out,
                                            _f32(y, "y"), _f32(pre, "pre"), C.c_void_p(_stream_ptr(stream))))
        return y, pre

    def mlp_backward(self, params, x, pre, dy, n_hid: int, n_out: int, grad=None, stream=None):
        B, n_in = int(x.shape[0]), int(x.shape[1])
        grad = torch.empty_like(params) if grad is None else grad
        self._check(self.lib.qc_mlp_backward(self.h, _f32(params, "params"), _f32(x, "x"), _f32(pre, "pre"),
                                             _f32(dy, "dy"), B, n_in, n_hid, n_out, _f32(grad, "grad"),
                                             C.c_void_p(_stream_ptr(stream))))
        return grad

    def adam_step(self, params, grad, m, v, lr: float, b1: float, b2: float, eps: float, step: int, stream=None):
        self._check(self.lib.qc_adam_step(self.h, _f32(params, "params"), _f32(grad, "grad"), _f32(m, "m"),
                                          _f32(v, "v"), int(params.numel()), float(lr), float(b1), float(b2),
                                          float(eps), int(step), C.c_void_p(_stream_ptr(stream))))

    def mse_grad(self, y, t, dy=None, loss=None, stream=None):
        dy = torch.empty_like(y) if dy is None else dy
        self._check(self.lib.qc_mse_grad(self.h, _f32(y, "y"), _f32(t, "t"), int(y.numel()), _f32(dy, "dy"),
                                         C.c_void_p(_ptr(loss, torch.float32, "loss")),
                                         C.c_void_p(_stream_ptr(stream))))
        return dy

    def ws_gains(self, y, n_ant: int, gains, stream=None):
        """qc_ws_gains: network output [n_int][n_ant*4] -> diagonal gains (complex128, in place)."""
        n_int = int(y.shape[0])
        if tuple(y.shape) != (n_int, n_ant * 4) or gains.numel() != n_int * n_ant * 4:
            raise ValueError("y must be [n_int][n_ant*4] and gains [.. n_int ..][n_ant][1][4]")
        self._check(self.lib.qc_ws_gains(self.h, _f32(y, "y"), n_int, int(n_ant),
                                         C.c_void_p(_ptr(gains, torch.complex128, "gains")),
                                         C.c_void_p(_stream_ptr(stream))))
        return gains

    def ws_labels(self, gains, n_ant: int, ref_ant: int = 0, y=None, stream=None):
        """qc_ws_labels: solved diagonal gains -> referenced targets [n_int][n_ant*4] (float32)."""
        n_int = gains.numel() // (n_ant * 4)
        y = torch.empty(n_int, n_ant * 4, dtype=torch.float32, device=gains.device) if y is None else y
        self._check(self.lib.qc_ws_labels(self.h, C.c_void_p(_ptr(gains, torch.complex128, "gains")), n_int,
                                          int(n_ant), int(ref_ant), C.c_void_p(_f32(y, "y")),
                                          C.c_void_p(_stream_ptr(stream))))
        return y

    def _out_like(self, vis, out):
        if out is None:
            out = torch.empty_like(vis.data)
        _ptr(out, vis.data.dtype, "out")
        if out.shape != vis.data.shape:
            raise ValueError("out must have the shape of data")
        return out

    @staticmethod
    def _mask(vis, dir_mask):
        if dir_mask is None:
            return None, None
        m = np.ascontiguousarray(np.asarray(dir_mask, dtype=np.uint8))
        if m.shape != (int(vis.model.shape[2]),):
            raise ValueError("dir_mask must have n_dir entries")
        return m, m.ctypes.data_as(C.c_void_p)

    def residual(self, vis, chain, dir_mask=None, out=None, stream=None) -> torch.Tensor:
        """qc_residual: D - sum_{d in mask} C_p M_d C_q^H."""
        out = self._out_like(vis, out)
        keep, mp = self._mask(vis, dir_mask)
        cv = _c_vis(vis)
        cc = _c_chain(chain)
        self._check(self.lib.qc_residual(self.h, C.byref(cv), cc, len(chain), mp, C.c_void_p(out.data_ptr()),
                                         C.c_void_p(_stream_ptr(stream))))
        return out

    def mad_flag(self, vis, resid, mode: str = "baseline", k: float = 5.0, flag_out=None, stats: bool = False,
                 stream=None):
        """qc_mad_flag: outlier flags from the residual by the median absolute
        deviation.  Returns (flags [n_row][n_chan] uint8, number of new flags,
        per-group (median, MAD) as a float64 tensor [n_groups][2] or None)."""
        if mode not in MAD_MODES:
            raise ValueError(f"unknown MAD mode {mode!r}")
        if not isinstance(resid, torch.Tensor) or resid.dtype != vis.data.dtype or not resid.is_contiguous() \
                or tuple(resid.shape) != tuple(vis.data.shape) or resid.device != vis.data.device:
            raise ValueError("resid must be a contiguous tensor shaped and typed like vis.data")
        if flag_out is None:
            flag_out = torch.empty_like(vis.flag)
        n_ant = int(vis.n_ant)
        n_groups = 1 if mode == "global" else max(1, n_ant * (n_ant - 1) // 2)
        st = torch.empty(n_groups, 2, dtype=torch.float64, device=vis.data.device) if stats else None
        n_new = C.c_int64(0)
        cv = _c_vis(vis)
        self._check(self.lib.qc_mad_flag(self.h, C.byref(cv), C.c_void_p(resid.data_ptr()), MAD_MODES[mode],
                                         float(k), C.c_void_p(_ptr(flag_out, torch.uint8, "flag_out")),
                                         C.c_void_p(st.data_ptr()) if st is not None else None,
                                         C.byref(n_new), C.c_void_p(_stream_ptr(stream))))
        return flag_out, int(n_new.value), st

    def interp_term(self, src, t_src, f_src, dst, t_dst, f_dst, n_ant: int, stream=None):
        """qc_interp_term: src's solutions onto dst's grid (dst's gains or params
        and gain flags written); coordinates are float64 device tensors."""
        cs = _c_chain([src])
        cd = _c_chain([dst])
        self._check(self.lib.qc_interp_term(self.h, cs, C.c_void_p(_ptr(t_src, torch.float64, "t_src")),
                                            C.c_void_p(_ptr(f_src, torch.float64, "f_src")), cd,
                                            C.c_void_p(_ptr(t_dst, torch.float64, "t_dst")),
                                            C.c_void_p(_ptr(f_dst, torch.float64, "f_dst")), int(n_ant),
                                            C.c_void_p(_stream_ptr(stream))))
        return dst

    def robust_weights(self, vis, resid, nu: float = 2.0, out=None, want_s2: bool = True, stream=None):
        """qc_robust_weights: Student's t weights from the residual; returns
        (weights like vis.weight, s2 or None when not asked for)."""
        if not isinstance(resid, torch.Tensor) or resid.dtype != vis.data.dtype or not resid.is_contiguous() \
                or tuple(resid.shape) != tuple(vis.data.shape) or resid.device != vis.data.device:
            raise ValueError("resid must be a contiguous tensor shaped and typed like vis.data")
        if out is None:
            out = torch.empty_like(vis.weight)
        if tuple(out.shape) != tuple(vis.weight.shape) or out.dtype != vis.weight.dtype:
            raise ValueError("out must be shaped and typed like vis.weight")
        s2 = C.c_double(0.0)
        cv = _c_vis(vis)
        self._check(self.lib.qc_robust_weights(self.h, C.byref(cv), C.c_void_p(resid.data_ptr()), float(nu),
                                               C.c_void_p(_ptr(out, vis.weight.dtype, "out")),
                                               C.byref(s2) if want_s2 else None, C.c_void_p(_stream_ptr(stream))))
        return out, (float(s2.value) if want_s2 else None)

    def corrected_weights(self, vis, chain, out=None, stream=None) -> torch.Tensor:
        """qc_corrected_weights: w |c_p,i|^2 |c_q,j|^2 (weights of the corrected data)."""
        if out is None:
            out = torch.empty_like(vis.weight)
        if tuple(out.shape) != tuple(vis.weight.shape) or out.dtype != vis.weight.dtype:
            raise ValueError("out must be shaped and typed like vis.weight")
        cv = _c_vis(vis)
        cc = _c_chain(chain)
        self._check(self.lib.qc_corrected_weights(self.h, C.byref(cv), cc, len(chain),
                                                  C.c_void_p(_ptr(out, vis.weight.dtype, "out")),
                                                  C.c_void_p(_stream_ptr(stream))))
        return out

    def predict(self, uvw, chan_freq, lm, stokes, spi, ref_freq, comp_dir, n_dir: int = 1, dtype: str = "c64",
                out=None, stream=None) -> torch.Tensor:
        """qc_predict_dft: model visibilities [n_row][n_chan][n_dir][4] from point
        components (device tensors: uvw [n_row][3] float64, chan_freq [n_chan]
        float64, lm [n_comp][2], stokes [n_comp][4], spi [n_comp], ref_freq
        [n_comp] float64, comp_dir [n_comp] int32)."""
        dev = uvw.device
        n_row, n_chan = int(uvw.shape[0]), int(chan_freq.shape[0])
        n_comp = int(lm.shape[0])
        cdt = {"c64": torch.complex64, "c128": torch.complex128}[dtype]
        if out is None:
            out = torch.empty(n_row, n_chan, n_dir, 4, dtype=cdt, device=dev)
        if tuple(out.shape) != (n_row, n_chan, n_dir, 4) or out.dtype != cdt:
            raise ValueError("out must be [n_row][n_chan][n_dir][4] of the requested dtype")
        if tuple(lm.shape) != (n_comp, 2) or tuple(stokes.shape) != (n_comp, 4) or spi.numel() != n_comp \
                or ref_freq.numel() != n_comp or comp_dir.numel() != n_comp or tuple(uvw.shape) != (n_row, 3):
            raise ValueError("inconsistent component or uvw shapes")
        sky = QcSky(n_comp=n_comp, lm=_ptr(lm, torch.float64, "lm"), stokes=_ptr(stokes, torch.float64, "stokes"),
                    spi=_ptr(spi, torch.float64, "spi"), ref_freq=_ptr(ref_freq, torch.float64, "ref_freq"),
                    dir=_ptr(comp_dir, torch.int32, "comp_dir"))
        self._check(self.lib.qc_predict_dft(self.h, C.c_void_p(_ptr(uvw, torch.float64, "uvw")), n_row,
                                            C.c_void_p(_ptr(chan_freq, torch.float64, "chan_freq")), n_chan,
                                            C.byref(sky), int(n_dir), {"c64": 0, "c128": 1}[dtype],
                                            C.c_void_p(_ptr(out, cdt, "out")), C.c_void_p(_stream_ptr(stream))))
        return out

    def apply(self, vis, chain, mode: str = "corrupt", dir_mask=None, out=None, stream=None) -> torch.Tensor:
        """qc_apply_gains: CORRUPT (model through the chain) or CORRECT (C_p^-1 D C_q^-H)."""
        out = self._out_like(vis, out)
        keep, mp = self._mask(vis, dir_mask)
        cv = _c_vis(vis)
        cc = _c_chain(chain)
        m = {"corrupt": 0, "correct": 1}[mode]
        self._check(self.lib.qc_apply_gains(self.h, C.byref(cv), cc, len(chain), m, mp,
                                            C.c_void_p(out.data_ptr()), C.c_void_p(_stream_ptr(stream))))
        return out


class Batch:
    """A qc_batch plan: many independent single-term problems solved by one
    graph launch (qc_batch_create / qc_batch_tune / qc_batch_run).

    problems: list of (vis, term) pairs, or (vis, term, chisq_ref) triples
    (chisq_ref: float64 per interval of the term, the warm-start fallback
    reference), with device tensors; each term's gains are solved in place on
    every run.  The plan keeps references to every tensor it was given."""

    def __init__(self, ctx: "Context", problems, tol: float = 1e-6, max_iter: int = 100,
                 prec: str = "mixed", damping: str = "auto", stream=None):
        self.ctx = ctx
        self.lib = ctx.lib
        self.problems = list(problems)
        self.stats = []
        arr = (QcProblem * len(self.problems))()
        for i, prob in enumerate(self.problems):
            vis, term = prob[0], prob[1]
            ref = prob[2] if len(prob) > 2 else None
            st = _stats_for(term, vis.data.device)
            self.stats.append(st)
            arr[i].vis = _c_vis(vis)
            arr[i].term = _c_chain([term])[0]
            arr[i].stats = _c_stats(st)
            if ref is not None:
                n_int = int(term.n_gt) * int(term.n_gf)
                if ref.numel() != n_int:
                    raise ValueError(f"problem {i}: chisq_ref needs {n_int} entries, got {ref.numel()}")
            arr[i].chisq_ref = _ptr(ref, torch.float64, "chisq_ref")
        self._arr = arr
        opts = QcSolveOpts(tol=float(tol), max_iter=int(max_iter), prec=PRECISIONS[prec],
                           damping=DAMPINGS[damping], stream=_stream_ptr(stream))
        h = C.c_void_p()
        ctx._check(self.lib.qc_batch_create(ctx.h, C.cast(arr, C.c_void_p), len(self.problems), C.byref(opts),
                                            C.byref(h)))
        self.h = h

    def tune(self, reps: int = 1):
        self.ctx._check(self.lib.qc_batch_tune(self.h, int(reps)))

    def run(self, stream=None):
        self.ctx._check(self.lib.qc_batch_run(self.h, C.c_void_p(_stream_ptr(stream))))

    def last_ms(self) -> float:
        return float(self.lib.qc_batch_last_ms(self.h))

    def n_intervals(self) -> int:
        """Solution intervals over every problem (rows of the per-interval arrays)."""
        return int(self.lib.qc_batch_n_intervals(self.h))

    def ws_features(self, feat: torch.Tensor, chisq_unit: Optional[torch.Tensor] = None, ref_ant: int = 0,
                    stream=None):
        """qc_batch_ws_features: feat [n_intervals][stride] float32, chisq_unit [n_intervals]
        float64 or None, rows in problem order."""
        if feat.dim() != 2 or feat.shape[0] != self.n_intervals():
            raise ValueError(f"feat must be [{self.n_intervals()}][stride], got {tuple(feat.shape)}")
        if chisq_unit is not None and chisq_unit.numel() != self.n_intervals():
            raise ValueError(f"chisq_unit needs {self.n_intervals()} entries")
        self.ctx._check(self.lib.qc_batch_ws_features(self.h, _ptr(feat, torch.float32, "feat"), int(feat.shape[1]),
                                                      _ptr(chisq_unit, torch.float64, "chisq_unit"), int(ref_ant),
                                                      _stream_ptr(stream)))

    def ws_gains(self, y: torch.Tensor, stream=None):
        """qc_batch_ws_gains: every problem's diagonal gains from y [n_intervals][stride] float32."""
        if y.dim() != 2 or y.shape[0] != self.n_intervals():
            raise ValueError(f"y must be [{self.n_intervals()}][stride], got {tuple(y.shape)}")
        self.ctx._check(self.lib.qc_batch_ws_gains(self.h, _ptr(y, torch.float32, "y"), int(y.shape[1]),
                                                   _stream_ptr(stream)))

    def schedule(self):
        n = BATCH_BUCKETS
        items, waves, rps = (C.c_int32 * n)(), (C.c_int32 * n)(), (C.c_int32 * n)()
        ms = (C.c_float * n)()
        self.ctx._check(self.lib.qc_batch_schedule(self.h, items, waves, rps, ms, n))
        return [dict(items=items[i], waves=waves[i], rows_per_step=rps[i], tuned_ms=float(ms[i]))
                for i in range(n)]

    def close(self):
        if getattr(self, "h", None):
            self.lib.qc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
