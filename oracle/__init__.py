"""Plain FP64 CPU oracle for the transient F-statistic map.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and this
package never imports the GPU library.  The arithmetic lives in
`tfstat_oracle.c` (direct summation per cell, FP64, libm exp); this module
only marshals numpy arrays through ctypes.

Every function takes the atoms and grid as plain arrays:
  ts      int64 [n_sft]           SFT start times, strictly increasing
  a2,b2,ab float64 [n_sft]
  fa, fb  float64 [n_bins, n_sft, 2]   (re, im)
  t0, tau int64 [n_t0], [n_tau]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build as _build, library_path

RECT = 0
EXP = 1

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    src = os.path.join(os.path.dirname(__file__), "tfstat_oracle.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        _build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int, ctypes.c_int64
    lib.tfo_fmap.argtypes = [i32, i32, P, P, P, P, i32, P, P, i32, P, i32, P, i32, P]
    lib.tfo_fmap.restype = i32
    lib.tfo_cells.argtypes = [i32, i32, P, P, P, P, i32, P, P, i32, P, i32, P,
                              i32, P, P, i32, P]
    lib.tfo_cells.restype = i32
    lib.tfo_cell_sums.argtypes = [i32, i32, P, P, P, P, i32, P, P, i64, i64, P]
    lib.tfo_cell_sums.restype = i32
    lib.tfo_reduce.argtypes = [P, i32, i64, P, P, P]
    lib.tfo_reduce.restype = i32
    lib.tfo_fmap_shape.argtypes = [P, i32, i64, i64] + lib.tfo_fmap.argtypes[1:]
    lib.tfo_fmap_shape.restype = i32
    lib.tfo_cells_shape.argtypes = [P, i32, i64, i64] + lib.tfo_cells.argtypes[1:]
    lib.tfo_cells_shape.restype = i32
    _lib = lib
    return lib


def _kind(kind) -> int:
    if kind in ("rect", RECT):
        return RECT
    if kind in ("exp", EXP):
        return EXP
    raise ValueError(f"unknown window kind {kind!r}")


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _i64(x):
    return np.ascontiguousarray(x, dtype=np.int64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _atoms_args(ts, a2, b2, ab, fa, fb):
    ts, a2, b2, ab = _i64(ts), _f64(a2), _f64(b2), _f64(ab)
    fa, fb = _f64(fa), _f64(fb)
    if fa.ndim == 2:
        fa = fa[None]
    if fb.ndim == 2:
        fb = fb[None]
    n = ts.shape[0]
    if not (a2.shape == b2.shape == ab.shape == (n,)):
        raise ValueError("a2, b2, ab must have shape [n_sft]")
    if fa.shape != fb.shape or fa.shape[1:] != (n, 2):
        raise ValueError("fa, fb must have shape [n_bins, n_sft, 2]")
    return ts, a2, b2, ab, fa, fb


def fmap(kind, ts, a2, b2, ab, fa, fb, t0, tau, n_threads: int = 0) -> np.ndarray:
    """Full 2F map, float64 [n_bins, n_t0, n_tau]."""
    lib = _load()
    ts, a2, b2, ab, fa, fb = _atoms_args(ts, a2, b2, ab, fa, fb)
    t0, tau = _i64(t0), _i64(tau)
    nb = fa.shape[0]
    out = np.empty((nb, t0.shape[0], tau.shape[0]), dtype=np.float64)
    rc = lib.tfo_fmap(_kind(kind), ts.shape[0], _ptr(ts), _ptr(a2), _ptr(b2), _ptr(ab),
                      nb, _ptr(fa), _ptr(fb), t0.shape[0], _ptr(t0), tau.shape[0],
                      _ptr(tau), int(n_threads), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return out


def fmap_shape(shape, support, ts, a2, b2, ab, fa, fb, t0, tau, n_threads: int = 0) -> np.ndarray:
    """Full 2F map for a general window shape: `shape` holds samples of
    s(x) evenly spaced over x in [0, num/den], support = (num, den); the window
    covers [t0, t0 + floor(tau * num / den))."""
    lib = _load()
    ts, a2, b2, ab, fa, fb = _atoms_args(ts, a2, b2, ab, fa, fb)
    t0, tau = _i64(t0), _i64(tau)
    sh = _f64(shape)
    nb = fa.shape[0]
    out = np.empty((nb, t0.shape[0], tau.shape[0]), dtype=np.float64)
    rc = lib.tfo_fmap_shape(_ptr(sh), sh.shape[0], int(support[0]), int(support[1]),
                            ts.shape[0], _ptr(ts), _ptr(a2), _ptr(b2), _ptr(ab),
                            nb, _ptr(fa), _ptr(fb), t0.shape[0], _ptr(t0), tau.shape[0],
                            _ptr(tau), int(n_threads), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return out


def cells_shape(shape, support, ts, a2, b2, ab, fa, fb, t0, tau, m_idx, n_idx,
                n_threads: int = 0) -> np.ndarray:
    """2F at selected cells for a general window shape, float64 [n_bins, n_sel]."""
    lib = _load()
    ts, a2, b2, ab, fa, fb = _atoms_args(ts, a2, b2, ab, fa, fb)
    t0, tau = _i64(t0), _i64(tau)
    sh = _f64(shape)
    mi = np.ascontiguousarray(m_idx, dtype=np.int32)
    ni = np.ascontiguousarray(n_idx, dtype=np.int32)
    nb = fa.shape[0]
    out = np.empty((nb, mi.shape[0]), dtype=np.float64)
    rc = lib.tfo_cells_shape(_ptr(sh), sh.shape[0], int(support[0]), int(support[1]),
                             ts.shape[0], _ptr(ts), _ptr(a2), _ptr(b2), _ptr(ab),
                             nb, _ptr(fa), _ptr(fb), t0.shape[0], _ptr(t0), tau.shape[0],
                             _ptr(tau), mi.shape[0], _ptr(mi), _ptr(ni), int(n_threads), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return out


def cells(kind, ts, a2, b2, ab, fa, fb, t0, tau, m_idx, n_idx,
          n_threads: int = 0) -> np.ndarray:
    """2F at selected cells, float64 [n_bins, n_sel]."""
    lib = _load()
    ts, a2, b2, ab, fa, fb = _atoms_args(ts, a2, b2, ab, fa, fb)
    t0, tau = _i64(t0), _i64(tau)
    mi = np.ascontiguousarray(m_idx, dtype=np.int32)
    ni = np.ascontiguousarray(n_idx, dtype=np.int32)
    nb = fa.shape[0]
    out = np.empty((nb, mi.shape[0]), dtype=np.float64)
    rc = lib.tfo_cells(_kind(kind), ts.shape[0], _ptr(ts), _ptr(a2), _ptr(b2), _ptr(ab),
                       nb, _ptr(fa), _ptr(fb), t0.shape[0], _ptr(t0), tau.shape[0],
                       _ptr(tau), mi.shape[0], _ptr(mi), _ptr(ni), int(n_threads),
                       _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return out


def cell_sums(kind, ts, a2, b2, ab, fa, fb, t0: int, tau: int):
    """Windowed sums of one cell: (A, B, C, F_a[n_bins] complex, F_b[n_bins])."""
    lib = _load()
    ts, a2, b2, ab, fa, fb = _atoms_args(ts, a2, b2, ab, fa, fb)
    nb = fa.shape[0]
    out = np.empty(3 + 4 * nb, dtype=np.float64)
    rc = lib.tfo_cell_sums(_kind(kind), ts.shape[0], _ptr(ts), _ptr(a2), _ptr(b2),
                           _ptr(ab), nb, _ptr(fa), _ptr(fb), int(t0), int(tau), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    f = out[3:].reshape(nb, 4)
    return out[0], out[1], out[2], f[:, 0] + 1j * f[:, 1], f[:, 2] + 1j * f[:, 3]


def reduce(twoF: np.ndarray):
    """Per-map (max2F, argmax linear index, logB) over the last two axes."""
    lib = _load()
    arr = _f64(twoF)
    if arr.ndim == 2:
        arr = arr[None]
    n_maps = arr.shape[0]
    n_cells = int(np.prod(arr.shape[1:]))
    mx = np.empty(n_maps, dtype=np.float64)
    am = np.empty(n_maps, dtype=np.int64)
    lb = np.empty(n_maps, dtype=np.float64)
    rc = lib.tfo_reduce(_ptr(arr), n_maps, n_cells, _ptr(mx), _ptr(am), _ptr(lb))
    if rc != 0:
        raise ValueError("oracle: invalid arguments")
    return mx, am, lb


def fmap_atoms(atoms, win, n_threads: int = 0) -> np.ndarray:
    """Convenience: full map from generator objects (tfsynth.Atoms, Window)."""
    if win.kind == "shape":
        return fmap_shape(win.shape, win.support, atoms.timestamps, atoms.a2, atoms.b2, atoms.ab,
                          atoms.fa, atoms.fb, win.t0, win.tau, n_threads)
    return fmap(win.kind, atoms.timestamps, atoms.a2, atoms.b2, atoms.ab,
                atoms.fa, atoms.fb, win.t0, win.tau, n_threads)


def cells_atoms(atoms, win, m_idx, n_idx, n_threads: int = 0) -> np.ndarray:
    """Convenience: 2F at cells (m_idx[i], n_idx[i]) from generator objects,
    float64 [n_bins, n_sel]."""
    if win.kind == "shape":
        return cells_shape(win.shape, win.support, atoms.timestamps, atoms.a2, atoms.b2, atoms.ab,
                           atoms.fa, atoms.fb, win.t0, win.tau, m_idx, n_idx, n_threads)
    return cells(win.kind, atoms.timestamps, atoms.a2, atoms.b2, atoms.ab,
                 atoms.fa, atoms.fb, win.t0, win.tau, m_idx, n_idx, n_threads)


def results(atoms, win, twoF: np.ndarray):
    """Per-bin result records {max2F, m, n, t0, tau, logB} from a full map."""
    mx, am, lb = reduce(twoF)
    out = []
    for b in range(twoF.shape[0]):
        m, n = divmod(int(am[b]), win.n_tau)
        out.append(dict(max2F=float(mx[b]), m=m, n=n, t0=int(win.t0[m]),
                        tau=int(win.tau[n]), logB=float(lb[b])))
    return out
