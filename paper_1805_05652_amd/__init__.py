"""tfstat: transient F-statistic maps on AMD MI355X.

Thin Python binding of the C ABI in include/tfstat.h (libtfstat.so).  Every
step of the map (slot planes, weight tables, windowed sums, D, 2F,
reductions) runs in the library's HIP kernels; this module only converts
arguments.  PyTorch supplies the device arena and the stream.

Method: Keitel & Ashton, arXiv:1805.05652 (section 2: windows and F from
windowed atom sums; section 3: the atoms-plus-grid inputs and the two window
kernels; appendix A footnote: the marginalised Bayes factor).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional

import numpy as np

from . import _abi
from ._abi import TfstatError  # noqa: F401

PRECISIONS = {"fp64": _abi.PREC_FP64, "fp32": _abi.PREC_FP32, "bf16x3": _abi.PREC_BF16X3,
              "recur64": _abi.PREC_RECUR64, "f16x3": _abi.PREC_F16X3}
WINDOWS = {"rect": _abi.WIN_RECT, "exp": _abi.WIN_EXP, "shape": _abi.WIN_SHAPE}


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


class _WindowArgs:
    """Keeps the window struct and its backing arrays alive for a call."""

    def __init__(self, kind, t0, tau, t0_regular=None, tau_regular=None, shape=None, support=(1, 1)):
        self.t0 = np.ascontiguousarray(t0, dtype=np.int64)
        self.tau = np.ascontiguousarray(tau, dtype=np.int64)
        self.shape = None if shape is None else np.ascontiguousarray(shape, dtype=np.float64)
        w = _abi.Window()
        w.type = WINDOWS[kind] if isinstance(kind, str) else int(kind)
        w.n_t0 = int(self.t0.shape[0])
        w.n_tau = int(self.tau.shape[0])
        w.reserved = 0
        if t0_regular is not None:
            w.t0_min, w.dt0 = int(t0_regular[0]), int(t0_regular[1])
            w.t0_list = None
        else:
            w.t0_list = self.t0.ctypes.data
        if tau_regular is not None:
            w.tau_min, w.dtau = int(tau_regular[0]), int(tau_regular[1])
            w.tau_list = None
        else:
            w.tau_list = self.tau.ctypes.data
        if self.shape is not None:
            w.shape = self.shape.ctypes.data
            w.n_shape = int(self.shape.shape[0])
            w.support_num, w.support_den = int(support[0]), int(support[1])
        self.struct = w

    @classmethod
    def from_window(cls, win):
        return cls(win.kind, win.t0, win.tau, getattr(win, "t0_regular", None),
                   getattr(win, "tau_regular", None), getattr(win, "shape", None),
                   getattr(win, "support", (1, 1)))


def _results(arr) -> List[dict]:
    return [dict(max2F=r.max2F, logB=r.logB, t0=int(r.t0), tau=int(r.tau), m=int(r.m), n=int(r.n))
            for r in arr]


class Context:
    """A library context on one GPU with a device arena owned by a torch tensor."""

    def __init__(self, device: int = 0, arena_bytes: int = 1 << 30, stream=None):
        import torch
        self._lib = _abi.load()
        self.device = int(device)
        self._torch = torch
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda:%d" % self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        _abi.check(self._lib.tfstat_ctx_create(self.device, ctypes.c_void_p(self.arena.data_ptr()),
                                               int(arena_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                               ctypes.byref(self._ctx)))
        self._bins = {}

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if self._ctx:
            _abi.check(self._lib.tfstat_ctx_destroy(self._ctx))
            self._ctx = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- atoms -------------------------------------------------------------------
    def upload(self, timestamps, a2, b2, ab, fa, fb, t_sft: int = 1800) -> int:
        ts = np.ascontiguousarray(timestamps, dtype=np.int64)
        a2 = np.ascontiguousarray(a2, dtype=np.float64)
        b2 = np.ascontiguousarray(b2, dtype=np.float64)
        ab = np.ascontiguousarray(ab, dtype=np.float64)
        fa = np.ascontiguousarray(fa, dtype=np.float64)
        fb = np.ascontiguousarray(fb, dtype=np.float64)
        if fa.ndim == 2:
            fa = fa[None]
            fb = fb[None]
        n = int(ts.shape[0])
        if a2.shape != (n,) or b2.shape != (n,) or ab.shape != (n,) or fa.shape[1:] != (n, 2) \
                or fb.shape != fa.shape:
            raise ValueError("atom arrays have inconsistent shapes")
        d = _abi.AtomsDesc()
        d.n_sft = n
        d.n_bins = int(fa.shape[0])
        d.t_sft = int(t_sft)
        d.timestamps = ts.ctypes.data
        d.a2, d.b2, d.ab = a2.ctypes.data, b2.ctypes.data, ab.ctypes.data
        d.fa, d.fb = fa.ctypes.data, fb.ctypes.data
        out = ctypes.c_uint64()
        _abi.check(self._lib.tfstat_atoms_upload(self._ctx, ctypes.byref(d), ctypes.byref(out)))
        self._bins[out.value] = d.n_bins
        return out.value

    def upload_atoms(self, atoms) -> int:
        """Uploads a tfsynth.Atoms object."""
        return self.upload(atoms.timestamps, atoms.a2, atoms.b2, atoms.ab, atoms.fa, atoms.fb,
                           atoms.t_sft)

    def free(self, atoms_id: int):
        _abi.check(self._lib.tfstat_atoms_free(self._ctx, ctypes.c_uint64(atoms_id)))
        self._bins.pop(atoms_id, None)

    def _n_bins(self, atoms_id: int) -> int:
        nb = self._bins.get(atoms_id)
        if nb is None:
            nb = self.atoms_info(atoms_id)[1]
        return nb

    def atoms_info(self, atoms_id: int):
        k = ctypes.c_int32()
        b = ctypes.c_int32()
        _abi.check(self._lib.tfstat_atoms_info(self._ctx, ctypes.c_uint64(atoms_id), ctypes.byref(k),
                                               ctypes.byref(b)))
        return k.value, b.value

    # -- maps --------------------------------------------------------------------
    def fmap(self, atoms_id: int, win, precision="fp32", want_map: bool = False,
             out=None):
        """Map of every bin over `win` (a tfsynth.Window-like object).

        Returns (per-bin result dicts, 2F map tensor [bins, n_t0, n_tau] or
        None).  `out` may be a preallocated float32 CUDA tensor for the map.
        """
        wa = _WindowArgs.from_window(win)
        nb = self._n_bins(atoms_id)
        res = (_abi.BinResult * nb)()
        twoF = out
        if want_map and twoF is None:
            twoF = self._torch.empty((nb, wa.struct.n_t0, wa.struct.n_tau), dtype=self._torch.float32,
                                     device="cuda:%d" % self.device)
        if twoF is not None:
            if twoF.dtype != self._torch.float32 or not twoF.is_contiguous() or \
                    twoF.numel() != nb * wa.struct.n_t0 * wa.struct.n_tau:
                raise ValueError("out must be a contiguous float32 tensor of bins*n_t0*n_tau")
            ptr = ctypes.c_void_p(twoF.data_ptr())
        else:
            ptr = None
        _abi.check(self._lib.tfstat_fmap(self._ctx, ctypes.c_uint64(atoms_id), ctypes.byref(wa.struct),
                                         _prec(precision), ptr, res))
        return _results(res), twoF

    def window_odds(self, atoms_id: int, win_a, win_b, precision="fp32") -> np.ndarray:
        """Per-bin log odds of window model a against b on the same atoms:
        logB_a - logB_b (tfstat_window_odds)."""
        wa = _WindowArgs.from_window(win_a)
        wb = _WindowArgs.from_window(win_b)
        out = np.empty(self._n_bins(atoms_id), dtype=np.float64)
        _abi.check(self._lib.tfstat_window_odds(self._ctx, ctypes.c_uint64(atoms_id), ctypes.byref(wa.struct),
                                                ctypes.byref(wb.struct), _prec(precision), out.ctypes.data))
        return out

    def logB(self, twoF) -> np.ndarray:
        """logB of each map of a float32 CUDA tensor [n_maps, n_t0, n_tau]."""
        t = twoF if twoF.dim() == 3 else twoF[None]
        if t.dtype != self._torch.float32 or not t.is_contiguous():
            raise ValueError("twoF must be a contiguous float32 tensor")
        out = np.empty(t.shape[0], dtype=np.float64)
        _abi.check(self._lib.tfstat_logB(self._ctx, ctypes.c_void_p(t.data_ptr()), int(t.shape[0]),
                                         int(t.shape[1]), int(t.shape[2]), out.ctypes.data))
        return out

    def logB_noalloc(self, twoF, out):
        """tfstat_logB_noalloc: logB of each map of a float32 CUDA tensor
        [n_maps, n_t0, n_tau] into `out`, a float64 CUDA tensor [n_maps],
        asynchronously on the context's stream and without any allocation."""
        t = twoF if twoF.dim() == 3 else twoF[None]
        if t.dtype != self._torch.float32 or not t.is_contiguous():
            raise ValueError("twoF must be a contiguous float32 tensor")
        if out.dtype != self._torch.float64 or not out.is_contiguous() or out.numel() != t.shape[0]:
            raise ValueError("out must be a contiguous float64 tensor of n_maps values")
        _abi.check(self._lib.tfstat_logB_noalloc(self._ctx, ctypes.c_void_p(t.data_ptr()), int(t.shape[0]),
                                                 int(t.shape[1]), int(t.shape[2]),
                                                 ctypes.c_void_p(out.data_ptr())))
        return out

    # -- serving -------------------------------------------------------------------
    def submit(self, atoms_id: int, win, precision="fp32") -> int:
        wa = _WindowArgs.from_window(win)
        t = ctypes.c_uint64()
        _abi.check(self._lib.tfstat_submit(self._ctx, ctypes.c_uint64(atoms_id), ctypes.byref(wa.struct),
                                           _prec(precision), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, n_bins: int) -> Optional[List[dict]]:
        """Results if the ticket finished (the ticket is then retired), else None."""
        res = (_abi.BinResult * n_bins)()
        done = ctypes.c_int()
        _abi.check(self._lib.tfstat_poll(self._ctx, ctypes.c_uint64(ticket), res, ctypes.byref(done)))
        return _results(res) if done.value else None

    def cancel(self, ticket: int):
        _abi.check(self._lib.tfstat_cancel(self._ctx, ctypes.c_uint64(ticket)))

    def serve_config(self, max_batch: int):
        """Requests admitted together into one fused batch, at most."""
        _abi.check(self._lib.tfstat_serve_config(self._ctx, int(max_batch)))

    def tiling_config(self, runs_min_spread: int = -1, split_min_bins: int = -1):
        """Exponential maps whose 64-row t0 tiles span at least
        runs_min_spread slots (median) use the runs form (0 = every map, -1 =
        automatic: when the span exceeds the band stage, except one-bin FP32
        maps); FP32 maps with at least split_min_bins bins use the split form
        (0 = never, -1 = default 8)."""
        _abi.check(self._lib.tfstat_tiling_config(self._ctx, int(runs_min_spread), int(split_min_bins)))

    # -- uneven batch ----------------------------------------------------------------
    def batch(self, items, precision="fp32", tune: bool = False, variant: str = None) -> "Batch":
        """Plans a batch of maps: items is a sequence of (atoms_id, window).
        variant (a name of Batch.stats()["variant"]) forces that fused-kernel
        build instead of the default or the autotuner's choice."""
        return Batch(self, items, precision, tune, variant)

    # -- profiling -----------------------------------------------------------------
    def profile(self, on: bool = True):
        _abi.check(self._lib.tfstat_profile_enable(self._ctx, 1 if on else 0))

    def profile_reset(self):
        _abi.check(self._lib.tfstat_profile_reset(self._ctx))

    def profile_read(self) -> dict:
        out = {}
        for k, name in enumerate(_abi.KERNEL_NAMES):
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            _abi.check(self._lib.tfstat_profile_read(self._ctx, k, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (n.value, ms.value)
        return out


class Batch:
    """Many maps planned together and run as one captured graph with one
    persistent fused launch (tfstat_batch_*)."""

    def __init__(self, ctx: Context, items, precision="fp32", tune: bool = False, variant: str = None):
        self._ctx = ctx
        self._lib = ctx._lib
        items = list(items)
        if not items:
            raise ValueError("a batch needs at least one map")
        self._wins = [_WindowArgs.from_window(w) for _, w in items]
        ids = (ctypes.c_uint64 * len(items))(*[int(a) for a, _ in items])
        wins = (_abi.Window * len(items))(*[w.struct for w in self._wins])
        self._bins = [ctx._n_bins(int(a)) for a, _ in items]
        self._h = ctypes.c_void_p()
        mode = 1 if tune else 0
        if variant is not None:
            mode = -1 - _abi.BATCH_VARIANTS.index(variant)
        _abi.check(self._lib.tfstat_batch_create(ctx._ctx, len(items), ids, wins, _prec(precision),
                                                 mode, ctypes.byref(self._h)))

    def run(self, timed: bool = False) -> List[List[dict]]:
        """Runs the batch (graph replay, or direct launches timing the fused
        kernel when timed); per map, the list of its per-bin result dicts."""
        res = (_abi.BinResult * sum(self._bins))()
        _abi.check(self._lib.tfstat_batch_run(self._ctx._ctx, self._h, 1 if timed else 0, res))
        out, o = [], 0
        for nb in self._bins:
            out.append(_results(res[o:o + nb]))
            o += nb
        return out

    def stats(self) -> dict:
        st = _abi.BatchStats()
        _abi.check(self._lib.tfstat_batch_stats_read(self._h, ctypes.byref(st)))
        return dict(variant=_abi.BATCH_VARIANTS[st.variant], groups=st.groups, n_tiles=st.n_tiles,
                    n_results=st.n_results, tune_ms=st.tune_ms, last_ms=st.last_ms,
                    last_fused_ms=st.last_fused_ms, last_mfma_ms=st.last_mfma_ms)

    def close(self):
        if self._h:
            _abi.check(self._lib.tfstat_batch_destroy(self._ctx._ctx, self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def version() -> str:
    return _abi.load().tfstat_version().decode()
