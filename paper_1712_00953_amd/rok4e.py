"""Python binding of librok4e.so (argument marshalling only).

Device memory and streams come from PyTorch: state arrays are float64 CUDA (ROCm)
tensors passed by data pointer, the stream is torch's current stream.  Every step of
the reaction substep runs in the HIP library; there is no fallback path, and loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ROK4E_LIB names another build of the same library (e.g. one compiled with different
# tuning macros); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("ROK4E_LIB") or os.path.join(HERE, "librok4e.so")

OK, EINVAL, ENOMEM, EHIP, ECAPTURE, ENOTSUP, ESTATIC = 0, -1, -2, -3, -4, -5, -6
STATIC_MAX_CELLS = 1 << 21
FP64, MIXED = 0, 1
PERSISTENT, PER_ATTEMPT = 0, 1
SPLIT_SIMPLER, SPLIT_STRANG = 0, 1
METHOD_ROK4E, METHOD_RKDP45 = 0, 1
ORDER_HOT_FIRST, ORDER_ARRAY = 0, 1
GATHER_AUTO, GATHER_LDS, GATHER_PRIVATE = 0, 1, 2
CELL_OK, CELL_MAX_ATTEMPTS, CELL_STEP_UNDERFLOW, CELL_BAD_INPUT = 0, 1, 2, 3

EXPORTS = ["rok4e_options_default", "rok4e_mech_create", "rok4e_mech_destroy", "rok4e_set_options",
           "rok4e_get_options", "rok4e_reserve", "rok4e_integrate", "rok4e_integrate_forced",
           "rok4e_integrate_ex", "rok4e_integrate_conservative", "rok4e_integrate_static",
           "rok4e_tune", "rok4e_rhs", "rok4e_arnoldi", "rok4e_transport", "rok4e_split_workspace_bytes",
           "rok4e_split_step", "rok4e_get_stats", "rok4e_cell_stats_ptr",
           "rok4e_copy_cell_stats", "rok4e_fma_probe", "rok4e_strerror"]


class MechDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("W", C.c_void_p), ("cp", C.c_void_p), ("hf", C.c_void_p),
                ("reac", C.c_void_p), ("prod", C.c_void_p),
                ("lnAf", C.c_void_p), ("bf", C.c_void_p), ("Ef", C.c_void_p),
                ("lnAr", C.c_void_p), ("br", C.c_void_p), ("Er", C.c_void_p),
                ("n_elements", C.c_int32), ("elem", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("M", C.c_int32), ("precision", C.c_int32), ("max_attempts", C.c_int32),
                ("fixed_steps", C.c_int32), ("lanes_per_cell", C.c_int32),
                ("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("scheduling", C.c_int32), ("method", C.c_int32), ("cell_order", C.c_int32),
                ("jvp_gather", C.c_int32), ("waves_per_simd", C.c_int32), ("h0", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("lanes_per_cell", C.c_int32), ("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("jvp_gather", C.c_int32), ("waves_per_simd", C.c_int32), ("ms", C.c_float),
                ("ms_default", C.c_float),
                ("candidates", C.c_int32), ("from_cache", C.c_int32)]


X_PERIODIC, X_INFLOW_OUTFLOW = 0, 1


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dx", C.c_double),
                ("vel", C.c_double), ("diff", C.c_double), ("x_boundary", C.c_int32),
                ("inflow", C.c_void_p)]


HIST_BINS = 22


class Stats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("accepted", C.c_int64), ("rejected", C.c_int64),
                ("max_attempts", C.c_int64), ("status_count", C.c_int64 * 4),
                ("attempt_histogram", C.c_int64 * HIST_BINS)]


class Rok4eError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


def load():
    """Loads librok4e.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950); there is no fallback implementation")
        lib = C.CDLL(LIB_PATH)
        vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double
        lib.rok4e_strerror.restype = C.c_char_p
        lib.rok4e_strerror.argtypes = [C.c_int]
        lib.rok4e_options_default.restype = None
        lib.rok4e_options_default.argtypes = [C.POINTER(Options)]
        lib.rok4e_mech_create.argtypes = [C.POINTER(MechDesc), C.POINTER(Options), C.POINTER(vp)]
        lib.rok4e_mech_destroy.argtypes = [vp]
        lib.rok4e_set_options.argtypes = [vp, C.POINTER(Options)]
        lib.rok4e_get_options.argtypes = [vp, C.POINTER(Options)]
        lib.rok4e_reserve.argtypes = [vp, i64]
        lib.rok4e_integrate.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, vp]
        lib.rok4e_integrate_forced.argtypes = [i64, vp, vp, vp, vp, vp, dbl, dbl, dbl, vp]
        lib.rok4e_integrate_ex.argtypes = [i64, vp, vp, vp, vp, vp, vp, dbl, dbl, dbl, vp]
        lib.rok4e_integrate_conservative.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, vp]
        lib.rok4e_integrate_static.argtypes = [i64, vp, vp, vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp]
        lib.rok4e_fma_probe.argtypes = [i64, C.c_int32, vp, vp]
        lib.rok4e_tune.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, C.c_int32, C.POINTER(TuneResult), vp]
        lib.rok4e_rhs.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp]
        lib.rok4e_transport.argtypes = [C.POINTER(Grid), C.c_int32, vp, vp, vp, vp]
        lib.rok4e_split_workspace_bytes.restype = C.c_size_t
        lib.rok4e_split_workspace_bytes.argtypes = [C.POINTER(Grid), C.c_int32]
        lib.rok4e_split_step.argtypes = [vp, C.POINTER(Grid), C.c_int32, vp, vp, vp, vp, dbl, dbl, dbl,
                                         C.c_int32, vp, C.c_size_t, vp]
        lib.rok4e_arnoldi.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.rok4e_get_stats.argtypes = [vp, C.POINTER(Stats), vp]
        lib.rok4e_cell_stats_ptr.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        lib.rok4e_copy_cell_stats.argtypes = [vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


def grid(nx, ny, nz, dx, vel, diff, inflow=None) -> Grid:
    """A periodic grid, or with inflow (a contiguous FP64 device tensor of ns + 1 values: the
    ghost state before x = 0) an open one along x (zero-gradient outflow).  The grid keeps a
    reference to the inflow tensor."""
    if inflow is None:
        return Grid(int(nx), int(ny), int(nz), float(dx), float(vel), float(diff), X_PERIODIC, None)
    _need(inflow, inflow.numel(), "inflow")
    g = Grid(int(nx), int(ny), int(nz), float(dx), float(vel), float(diff), X_INFLOW_OUTFLOW, _ptr(inflow))
    g.inflow_tensor = inflow
    return g


def _need_inflow(g: Grid, n_species):
    if g.x_boundary == X_INFLOW_OUTFLOW:
        t = getattr(g, "inflow_tensor", None)
        if t is not None and t.numel() != int(n_species) + 1:
            raise ValueError(f"inflow: {t.numel()} values, expected n_species + 1 = {int(n_species) + 1}")


def transport(g: Grid, n_species, Y, T, S, stream=None):
    """rok4e_transport: S[r * n + c] = T(U)_r for the state (Y, T) on grid g."""
    n = int(g.nx) * int(g.ny) * int(g.nz)
    for t, rows, name in ((Y, int(n_species), "Y"), (T, 1, "T"), (S, int(n_species) + 1, "S")):
        _need(t, rows * n, name, rows=rows)
    _need_inflow(g, n_species)
    _check(load().rok4e_transport(C.byref(g), int(n_species), _ptr(Y), _ptr(T), _ptr(S), _stream(stream)),
           "rok4e_transport")


def fma_probe(out, iters, stream=None):
    """rok4e_fma_probe: out.numel() threads (a multiple of 256) each run iters rounds of
    eight FP64 FMA chains; 16 * out.numel() * iters operations."""
    _need(out, out.numel(), "out")
    _check(load().rok4e_fma_probe(int(out.numel()), int(iters), _ptr(out), _stream(stream)), "rok4e_fma_probe")


def strerror(code: int) -> str:
    return load().rok4e_strerror(int(code)).decode()


def _check(rc, what):
    if rc != OK:
        raise Rok4eError(rc, what)


def options(M=4, precision=FP64, max_attempts=0, fixed_steps=0, lanes_per_cell=0,
            waves_per_block=0, blocks_per_cu=0, scheduling=PERSISTENT, method=METHOD_ROK4E,
            h0=0.0, cell_order=None, jvp_gather=GATHER_AUTO, waves_per_simd=0) -> Options:
    order = ORDER_HOT_FIRST if cell_order is None else int(cell_order)
    return Options(int(M), int(precision), int(max_attempts), int(fixed_steps), int(lanes_per_cell),
                   int(waves_per_block), int(blocks_per_cu), int(scheduling), int(method), order,
                   int(jvp_gather), int(waves_per_simd), float(h0))


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return C.c_void_p(t.data_ptr())
    return C.c_void_p(int(t))


def _need(t, count, name, dtype="float64", rows=None):
    """Host-side check of a device operand before its pointer goes to a kernel: of the
    given dtype, contiguous, on a GPU, at least count elements (the kernels index it up
    to there).  With rows, the operand is a structure-of-arrays block indexed
    [r * n + c] for n = count / rows cells: it must have exactly the shape (rows, n),
    or (n,) for rows == 1, or be flat with rows * n elements, so that a cell-major
    [n, rows] tensor or a wider [rows, N > n] one is refused instead of being read with
    the wrong stride."""
    if t is None:
        return
    if not hasattr(t, "data_ptr"):
        raise TypeError(f"{name}: expected a device tensor")
    import torch
    want = getattr(torch, dtype)
    if t.dtype != want or not t.is_cuda or not t.is_contiguous() or t.numel() < count:
        raise ValueError(f"{name}: need a contiguous {dtype} device tensor with >= {count} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    if rows is not None:
        n = count // rows if rows else 0
        shape = tuple(t.shape)
        ok = shape == (rows, n) or shape == (rows * n,) or (rows == 1 and shape == (n,))
        if not ok:
            raise ValueError(f"{name}: need shape ({rows}, {n}) (structure of arrays, stride {n}) "
                             f"or a flat tensor of {rows * n} elements, got {shape}")


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mech:
    """A mechanism handle on the current device (rok4e_mech_create)."""

    def __init__(self, mech, opts: Options | None = None, **kw):
        lib = load()
        self._arrays = [np.ascontiguousarray(a) for a in (
            np.asarray(mech.W, np.float64), np.asarray(mech.cp, np.float64), np.asarray(mech.hf, np.float64),
            np.asarray(mech.reac, np.int32).reshape(-1), np.asarray(mech.prod, np.int32).reshape(-1),
            np.asarray(mech.lnAf, np.float64), np.asarray(mech.bf, np.float64), np.asarray(mech.Ef, np.float64),
            np.asarray(mech.lnAr, np.float64), np.asarray(mech.br, np.float64), np.asarray(mech.Er, np.float64))]
        self.n_species = int(mech.n_species)
        self.n_reactions = int(mech.n_reactions)
        elem = getattr(mech, "elem", None)
        self._elem = None if elem is None else np.ascontiguousarray(np.asarray(elem, np.int8))
        n_el = 0 if self._elem is None else int(self._elem.shape[1])
        desc = MechDesc(self.n_species, self.n_reactions, *[a.ctypes.data for a in self._arrays],
                        n_el, None if self._elem is None else self._elem.ctypes.data)
        self.opts = opts if opts is not None else options(**kw)
        h = C.c_void_p()
        _check(lib.rok4e_mech_create(C.byref(desc), C.byref(self.opts), C.byref(h)), "rok4e_mech_create")
        self._h = h
        self.n_last = 0

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().rok4e_mech_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, opts: Options | None = None, **kw):
        o = opts if opts is not None else options(**kw)
        _check(load().rok4e_set_options(self._h, C.byref(o)), "rok4e_set_options")
        self.opts = o

    def get_options(self) -> Options:
        o = Options()
        _check(load().rok4e_get_options(self._h, C.byref(o)), "rok4e_get_options")
        return o

    def reserve(self, n_cells: int):
        _check(load().rok4e_reserve(self._h, int(n_cells)), "rok4e_reserve")

    def integrate(self, Y, T, p, dt, rtol, atol, S=None, stream=None, n_cells=None, h=None):
        """In-place integration of Y [ns, n], T [n] (float64 device tensors) over dt.
        h (float64 device tensor [n], optional): per-cell first trial steps in, the steps
        to start the next call from out (rok4e_integrate_ex)."""
        n = int(T.shape[0]) if n_cells is None else int(n_cells)
        ns = self.n_species
        for t, rows, name in ((Y, ns, "Y"), (T, 1, "T"), (p, 1, "p"), (S, ns + 1, "S"), (h, 1, "h")):
            _need(t, rows * n, name, rows=rows)
        rc = load().rok4e_integrate_ex(n, self._h, _ptr(Y), _ptr(T), _ptr(p), _ptr(S), _ptr(h), float(dt),
                                       float(rtol), float(atol), _stream(stream))
        _check(rc, "rok4e_integrate")
        self.n_last = n

    def integrate_static(self, Y, T, p, dt, rtol, atol, acc, rej, status, S=None, stream=None,
                         n_cells=None):
        """rok4e_integrate_static: as integrate (forcing S optional), allocating nothing;
        the per-cell accepted / rejected counts and status go to the int32 device tensors
        acc, rej, status [n]."""
        n = int(T.shape[0]) if n_cells is None else int(n_cells)
        ns = self.n_species
        for t, rows, name in ((Y, ns, "Y"), (T, 1, "T"), (p, 1, "p"), (S, ns + 1, "S")):
            _need(t, rows * n, name, rows=rows)
        for t, name in ((acc, "acc"), (rej, "rej"), (status, "status")):
            if n > 0 and t is None:
                raise ValueError(f"{name}: required")
            _need(t, n, name, "int32", rows=1)
        rc = load().rok4e_integrate_static(n, self._h, _ptr(Y), _ptr(T), _ptr(p), _ptr(S), float(dt),
                                           float(rtol), float(atol), _ptr(acc), _ptr(rej), _ptr(status),
                                           _stream(stream))
        _check(rc, "rok4e_integrate_static")

    def integrate_conservative(self, U, dt, rtol, atol, S=None, T_aux=None, stream=None, n_cells=None):
        """In-place reaction substep of the conservative variables U [(ns+5), n] (float64
        device tensor: rho Y_k, rho, rho u (3), rho E) with the auxiliary temperature;
        S: balancing constants of the same shape, T_aux [n]: the final auxiliary
        temperatures (rok4e_integrate_conservative)."""
        n = int(U.shape[-1]) if n_cells is None else int(n_cells)
        ns = self.n_species
        for t, rows, name in ((U, ns + 5, "U"), (S, ns + 5, "S"), (T_aux, 1, "T_aux")):
            _need(t, rows * n, name, rows=rows)
        rc = load().rok4e_integrate_conservative(n, self._h, _ptr(U), _ptr(S), _ptr(T_aux), float(dt),
                                                 float(rtol), float(atol), _stream(stream))
        _check(rc, "rok4e_integrate_conservative")
        self.n_last = n

    def tune(self, Y, T, p, dt, rtol, atol, force=False, stream=None) -> dict:
        """rok4e_tune: times the candidate launch layouts on a copy of this batch (or takes
        the cached choice for this mechanism size, M, precision and method) and keeps the
        fastest in the handle's options; returns the outcome as a dict."""
        n = int(T.shape[0])
        for t, rows, name in ((Y, self.n_species, "Y"), (T, 1, "T"), (p, 1, "p")):
            _need(t, rows * n, name, rows=rows)
        r = TuneResult()
        _check(load().rok4e_tune(n, self._h, _ptr(Y), _ptr(T), _ptr(p), float(dt), float(rtol), float(atol),
                                 int(bool(force)), C.byref(r), _stream(stream)), "rok4e_tune")
        self.opts = self.get_options()
        return {k: getattr(r, k) for k, _ in TuneResult._fields_}

    def rhs(self, Y, T, p, dY, dT, stream=None):
        n = int(T.shape[0])
        ns = self.n_species
        for t, rows, name in ((Y, ns, "Y"), (T, 1, "T"), (p, 1, "p"), (dY, ns, "dY"), (dT, 1, "dT")):
            _need(t, rows * n, name, rows=rows)
        _check(load().rok4e_rhs(n, self._h, _ptr(Y), _ptr(T), _ptr(p), _ptr(dY), _ptr(dT), _stream(stream)),
               "rok4e_rhs")

    def arnoldi(self, Y, T, p, Q, H, Meff, stream=None):
        n = int(T.shape[0])
        ns, M = self.n_species, int(self.opts.M)
        for t, rows, name in ((Y, ns, "Y"), (T, 1, "T"), (p, 1, "p")):
            _need(t, rows * n, name, rows=rows)
        for t, cnt, name in ((Q, n * M * (ns + 1), "Q"), (H, n * M * M, "H")):
            _need(t, cnt, name)
        _need(Meff, n, "Meff", "int32", rows=1)
        _check(load().rok4e_arnoldi(n, self._h, _ptr(Y), _ptr(T), _ptr(p), _ptr(Q), _ptr(H), _ptr(Meff),
                                    _stream(stream)), "rok4e_arnoldi")

    def split_step(self, grid: Grid, scheme, Y, T, p, h, rtol, atol, work, src=None, nsub=1, stream=None):
        """rok4e_split_step: one Simpler (or Strang) step of size h on the grid, in place.
        work: a device tensor of at least workspace_bytes(grid) bytes."""
        n = int(grid.nx) * int(grid.ny) * int(grid.nz)
        ns = self.n_species
        for t, rows, name in ((Y, ns, "Y"), (T, 1, "T"), (p, 1, "p"), (src, ns + 1, "src")):
            _need(t, rows * n, name, rows=rows)
        _need_inflow(grid, ns)
        _check(load().rok4e_split_step(self._h, C.byref(grid), int(scheme), _ptr(Y), _ptr(T), _ptr(p), _ptr(src),
                                       float(h), float(rtol), float(atol), int(nsub), _ptr(work),
                                       int(work.numel() * work.element_size()), _stream(stream)),
               "rok4e_split_step")
        self.n_last = n

    def workspace_bytes(self, grid: Grid) -> int:
        return int(load().rok4e_split_workspace_bytes(C.byref(grid), self.n_species))

    def stats(self, stream=None) -> dict:
        s = Stats()
        _check(load().rok4e_get_stats(self._h, C.byref(s), _stream(stream)), "rok4e_get_stats")
        return dict(n_cells=s.n_cells, accepted=s.accepted, rejected=s.rejected,
                    max_attempts=s.max_attempts, status_count=list(s.status_count),
                    attempt_histogram=list(s.attempt_histogram))

    def cell_stats(self, acc, rej, status, stream=None):
        """Copies per-cell counts of the last call into int32 tensors (host or device)."""
        _check(load().rok4e_copy_cell_stats(self._h, _ptr(acc), _ptr(rej), _ptr(status), _stream(stream)),
               "rok4e_copy_cell_stats")
