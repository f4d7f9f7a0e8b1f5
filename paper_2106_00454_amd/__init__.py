"""MI355X (gfx950) wave-packet continuum discretisation (WPCD) library.

Thin ctypes binding of ``libwpcd.so`` (C ABI in ``include/wpcd.h``).  This
module only marshals arguments: every step of the computation runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  If the
library has not been built, every entry point raises ``RuntimeError`` -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwpcd.so")

WPCD_OK = 0
WPCD_ERR_INVALID = -1
WPCD_ERR_NOMEM = -2
WPCD_ERR_DEVICE = -3
WPCD_ERR_NOCONV = -4
WPCD_ERR_AGAIN = -5
WPCD_ERR_BUSY = -6
WPCD_ERR_NUMERIC = -7
WPCD_ERR_UNSUPPORTED = -8

MIXED = 0
F64 = 1
DTYPE_F32 = 0
DTYPE_F64 = 1
PACKET_MOMENTUM = 0
PACKET_ENERGY = 1

#: every symbol declared in include/wpcd.h
EXPORTS = ("wpcd_create", "wpcd_destroy", "wpcd_last_error", "wpcd_version", "wpcd_grid_create",
           "wpcd_grid_create_packets", "wpcd_sigma_band", "wpcd_run", "wpcd_graph_create", "wpcd_graph_launch",
           "wpcd_graph_nodes", "wpcd_graph_destroy", "wpcd_autotune",
           "wpcd_grid_nodes", "wpcd_batch_create", "wpcd_batch_destroy", "wpcd_batch_layout_get",
           "wpcd_batch_offsets", "wpcd_basis_register", "wpcd_project", "wpcd_project_affine", "wpcd_eigh",
           "wpcd_eigh_noalloc",
           "wpcd_tmatrix", "wpcd_observables", "wpcd_sigma_tot", "wpcd_saclay", "wpcd_server_create", "wpcd_server_destroy",
           "wpcd_submit", "wpcd_poll", "wpcd_server_stats_get", "wpcd_profile_enable", "wpcd_stage_times",
           "wpcd_jacobi_counts", "wpcd_batch_jacobi_launches", "wpcd_mi_create", "wpcd_mi_destroy",
           "wpcd_mi_points", "wpcd_mi_layout_get", "wpcd_mi_solve")

STAGES = ("project", "jacobi_f32", "jacobi_f64", "refine", "tmatrix", "observables", "sigma", "warm_prep")


class WPCDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wpcd error {code}: {msg}")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("jacobi_tol_f32", ctypes.c_double), ("jacobi_tol_f64", ctypes.c_double),
                ("jacobi_block", ctypes.c_int32), ("refine_close_log10", ctypes.c_int32),
                ("jacobi_stop_f32", ctypes.c_double), ("jacobi_start", ctypes.c_int32),
                ("refine_gemm", ctypes.c_int32), ("refine_rr_steps", ctypes.c_int32)]


class _Item(ctypes.Structure):
    _fields_ = [("grid_id", ctypes.c_int32), ("n_ch", ctypes.c_int32), ("J", ctypes.c_int32),
                ("sample_id", ctypes.c_int32), ("basis_id", ctypes.c_int32), ("S", ctypes.c_int32),
                ("l", ctypes.c_int32)]


class _Layout(ctypes.Structure):
    _fields_ = [("u_elems", ctypes.c_int64), ("v_elems", ctypes.c_int64), ("eval_elems", ctypes.c_int64),
                ("t_doubles", ctypes.c_int64), ("delta_elems", ctypes.c_int64), ("mix_elems", ctypes.c_int64),
                ("coef_elems", ctypes.c_int64), ("n_items", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("max_n", ctypes.c_int32), ("max_nbins", ctypes.c_int32)]


class _MiItem(ctypes.Structure):
    _fields_ = [("n_ch", ctypes.c_int32), ("J", ctypes.c_int32), ("sample_id", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class _MiLayout(ctypes.Structure):
    _fields_ = [("u_elems", ctypes.c_int64), ("kmat_elems", ctypes.c_int64), ("delta_elems", ctypes.c_int64),
                ("mix_elems", ctypes.c_int64), ("n_items", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_q", ctypes.c_int32), ("n_e", ctypes.c_int32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch_items", ctypes.c_int32), ("max_queue", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _ReqChannel(ctypes.Structure):
    _fields_ = [("basis_id", ctypes.c_int32), ("J", ctypes.c_int32), ("coef_host", ctypes.c_void_p)]


class _Request(ctypes.Structure):
    _fields_ = [("channels_host", ctypes.POINTER(_ReqChannel)), ("n_channels", ctypes.c_int32),
                ("n_tlab", ctypes.c_int32), ("tlab_host", ctypes.c_void_p), ("sigma_host", ctypes.c_void_p),
                ("delta_host", ctypes.c_void_p), ("mix_host", ctypes.c_void_p), ("status_host", ctypes.c_void_p)]


class _PathArgs(ctypes.Structure):
    _fields_ = [("u_fine", ctypes.c_void_p), ("u_dtype", ctypes.c_int32), ("n_tlab", ctypes.c_int32),
                ("coef", ctypes.c_void_p), ("v64", ctypes.c_void_p), ("eval", ctypes.c_void_p),
                ("evec", ctypes.c_void_p), ("eig_status", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("t_status", ctypes.c_void_p), ("delta_deg", ctypes.c_void_p), ("mix_deg", ctypes.c_void_p),
                ("s_dev", ctypes.c_void_p), ("tlab_mev", ctypes.c_void_p), ("sigma_mb", ctypes.c_void_p)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("jacobi_block", ctypes.c_int32), ("refine_gemm", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("n_cand", ctypes.c_int32), ("best_ms", ctypes.c_double), ("cand_ms", ctypes.c_double * 4)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("items", ctypes.c_int64), ("peak_arena_bytes", ctypes.c_int64), ("queued", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("jacobi_launches", ctypes.c_int64), ("jacobi_sweeps", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises RuntimeError if libwpcd.so is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2106_00454_amd.build` "
                           "(there is no CPU fallback)")
    # torch first: its HIP runtime (same soname as the system one) must be the
    # one the process loads, so that torch's device memory and streams and the
    # library's kernels share one runtime
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "wpcd_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(_Config)]),
        "wpcd_destroy": (None, [vp]),
        "wpcd_last_error": (ctypes.c_char_p, []),
        "wpcd_version": (ctypes.c_char_p, []),
        "wpcd_grid_create": (i32, [vp, ctypes.POINTER(ctypes.c_double), i32, i32, ctypes.POINTER(i32)]),
        "wpcd_grid_create_packets": (i32, [vp, ctypes.POINTER(ctypes.c_double), i32, i32, i32, ctypes.POINTER(i32)]),
        "wpcd_sigma_band": (i32, [vp, dp, dp, dp, i32, dp, i32, dp, dp, vp]),
        "wpcd_run": (i32, [vp, ctypes.POINTER(_PathArgs), i32, vp]),
        "wpcd_graph_create": (i32, [vp, ctypes.POINTER(_PathArgs), i32, ctypes.POINTER(vp)]),
        "wpcd_graph_launch": (i32, [vp, vp]),
        "wpcd_graph_nodes": (i32, [vp, ctypes.POINTER(i64)]),
        "wpcd_graph_destroy": (None, [vp]),
        "wpcd_autotune": (i32, [vp, ctypes.POINTER(_PathArgs), i32, i32, ctypes.c_char_p,
                                ctypes.POINTER(_TuneResult), vp]),
        "wpcd_grid_nodes": (i32, [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "wpcd_batch_create": (i32, [vp, ctypes.POINTER(_Item), i32, ctypes.POINTER(vp)]),
        "wpcd_batch_destroy": (None, [vp]),
        "wpcd_batch_layout_get": (i32, [vp, ctypes.POINTER(_Layout)]),
        "wpcd_batch_offsets": (i32, [vp] + [ctypes.POINTER(i64)] * 7),
        "wpcd_basis_register": (i32, [vp, i32, i32, i32, dp, i32, vp, ctypes.POINTER(i32)]),
        "wpcd_project": (i32, [vp, dp, i32, dp, vp]),
        "wpcd_project_affine": (i32, [vp, dp, dp, vp]),
        "wpcd_eigh": (i32, [vp, dp, i32, dp, dp, dp, vp]),
        "wpcd_eigh_noalloc": (i32, [vp, dp, i32, dp, dp, dp, vp]),
        "wpcd_tmatrix": (i32, [vp, dp, dp, dp, i32, dp, dp, vp]),
        "wpcd_observables": (i32, [vp, dp, dp, dp, dp, vp]),
        "wpcd_sigma_tot": (i32, [vp, dp, dp, dp, i32, dp, vp]),
        "wpcd_saclay": (i32, [vp, dp, dp, dp, i32, dp, i32, dp, dp, vp]),
        "wpcd_server_create": (i32, [vp, ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]),
        "wpcd_server_destroy": (None, [vp]),
        "wpcd_submit": (i32, [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]),
        "wpcd_poll": (i32, [vp, ctypes.c_uint64]),
        "wpcd_server_stats_get": (i32, [vp, ctypes.POINTER(_ServerStats)]),
        "wpcd_profile_enable": (i32, [vp, i32]),
        "wpcd_stage_times": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        "wpcd_jacobi_counts": (i32, [vp, ctypes.POINTER(i64)]),
        "wpcd_batch_jacobi_launches": (i32, [vp, i32, ctypes.POINTER(i64)]),
        "wpcd_mi_create": (i32, [vp, ctypes.POINTER(_MiItem), i32, i32, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(vp)]),
        "wpcd_mi_destroy": (None, [vp]),
        "wpcd_mi_points": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "wpcd_mi_layout_get": (i32, [vp, ctypes.POINTER(_MiLayout)] + [ctypes.POINTER(i64)] * 4),
        "wpcd_mi_solve": (i32, [vp, dp, dp, dp, dp, dp, dp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code: int) -> None:
    if code != WPCD_OK:
        raise WPCDError(code, lib().wpcd_last_error().decode())


def version() -> str:
    return lib().wpcd_version().decode()


def _ptr(t, dtype, numel, name):
    """Device pointer of a contiguous CUDA tensor with at least numel elements."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: needs {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class Grid:
    id: int
    k_bounds: np.ndarray
    n_gauss: int
    nodes: np.ndarray
    weights: np.ndarray

    @property
    def n_wp(self) -> int:
        return self.k_bounds.size - 1


class Context:
    def __init__(self, device: int = 0, max_sweeps: int = 30, refine_steps: int = 2,
                 jacobi_tol_f32: float = 2e-7, jacobi_tol_f64: float = 1e-15, jacobi_block: int = 0,
                 refine_close_log10: int = 0, jacobi_stop_f32: float = 0.0, jacobi_start: int = 0,
                 refine_gemm: int = 0, refine_rr_steps: int = 0):
        L = lib()
        cfg = _Config(max_sweeps, refine_steps, jacobi_tol_f32, jacobi_tol_f64, jacobi_block, refine_close_log10,
                      jacobi_stop_f32, jacobi_start, refine_gemm, refine_rr_steps)
        h = ctypes.c_void_p()
        _check(L.wpcd_create(ctypes.byref(h), device, ctypes.byref(cfg)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().wpcd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid(self, k_bounds, n_gauss: int = 8, packet: int = PACKET_MOMENTUM) -> Grid:
        """Register a bin grid of momentum (default) or energy wave packets."""
        k = np.ascontiguousarray(k_bounds, dtype=np.float64)
        gid = ctypes.c_int()
        _check(lib().wpcd_grid_create_packets(self._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              k.size - 1, n_gauss, packet, ctypes.byref(gid)))
        m = (k.size - 1) * n_gauss
        nodes, weights = np.empty(m), np.empty(m)
        _check(lib().wpcd_grid_nodes(self._h, gid.value, nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     weights.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return Grid(gid.value, k, n_gauss, nodes, weights)

    def profile(self, on: bool = True) -> None:
        """Enable (and reset) or disable the library's per-stage event timers."""
        _check(lib().wpcd_profile_enable(self._h, 1 if on else 0))

    def stage_times(self) -> dict:
        """{stage: (total_ms, launches)} accumulated since profile(True)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(lib().wpcd_stage_times(self._h, ms, n))
        return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}

    def jacobi_counts(self) -> dict:
        """LDS Jacobi work since profile(True): rotations, pair visits, norm multiply-adds."""
        c = (ctypes.c_int64 * 3)()
        _check(lib().wpcd_jacobi_counts(self._h, c))
        return {"rotations": c[0], "pair_visits": c[1], "norm_madds": c[2]}

    def basis(self, grid: Grid, n_ch: int, terms, stream=None) -> "Basis":
        """Register the projections of fine-mesh terms U_t (a list of host (M, M)
        matrices, or a contiguous CUDA tensor of n_terms*M*M elements) for
        affine potentials U = sum_t c_t U_t on `grid` with n_ch channels."""
        import torch
        m = n_ch * grid.n_wp * grid.n_gauss
        if isinstance(terms, torch.Tensor):
            u = terms
            n_terms = u.numel() // (m * m)
        else:
            n_terms = len(terms)
            u = torch.empty(n_terms * m * m, dtype=torch.float64, device=f"cuda:{self.device}")
            for t, a in enumerate(terms):
                a = np.asarray(a, dtype=np.float64)
                if a.shape != (m, m):
                    raise ValueError(f"term {t}: expected shape {(m, m)}, got {a.shape}")
                u[t * m * m:(t + 1) * m * m].copy_(torch.from_numpy(a.ravel()))
        dt = DTYPE_F32 if u.dtype == torch.float32 else DTYPE_F64
        bid = ctypes.c_int()
        _check(lib().wpcd_basis_register(self._h, grid.id, n_ch, n_terms, _ptr(u, u.dtype, n_terms * m * m, "terms"),
                                         dt, _stream(stream), ctypes.byref(bid)))
        return Basis(bid.value, grid, n_ch, n_terms)

    def batch(self, items) -> "Batch":
        """items: iterable of (grid, n_ch, J, sample_id[, basis[, S, l]]) (basis None:
        fine-mesh input; S, l: total spin and first orbital momentum, needed by
        Batch.saclay only)."""
        return Batch(self, list(items))


@dataclass
class Basis:
    id: int
    grid: Grid
    n_ch: int
    n_terms: int


class Batch:
    def __init__(self, ctx: Context, items):
        self.ctx = ctx
        arr = (_Item * len(items))()
        self.grids = []
        self.items = []
        for i, spec in enumerate(items):
            g, n_ch, J, sid = spec[:4]
            basis = spec[4] if len(spec) > 4 else None
            S, l = (spec[5], spec[6]) if len(spec) > 6 else (-1, -1)
            arr[i] = _Item(g.id, n_ch, J, sid, -1 if basis is None else basis.id, S, l)
            self.grids.append(g)
            self.items.append((g, n_ch, J, sid))
        self.bases = [spec[4] if len(spec) > 4 else None for spec in items]
        h = ctypes.c_void_p()
        _check(lib().wpcd_batch_create(ctx._h, arr, len(items), ctypes.byref(h)))
        self._h = h
        lay = _Layout()
        _check(lib().wpcd_batch_layout_get(h, ctypes.byref(lay)))
        self.layout = {f: getattr(lay, f) for f, _ in _Layout._fields_}
        offs = [np.zeros(len(items), dtype=np.int64) for _ in range(7)]
        _check(lib().wpcd_batch_offsets(h, *[o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for o in offs]))
        self.u_off, self.v_off, self.eval_off, self.t_off, self.delta_off, self.mix_off, self.coef_off = offs

    def close(self):
        if getattr(self, "_h", None):
            lib().wpcd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ buffers
    def alloc(self, device="cuda"):
        """Output buffers of the whole path as torch tensors on `device`."""
        import torch
        L = self.layout
        f64 = dict(dtype=torch.float64, device=device)
        return {
            "v64": torch.empty(L["v_elems"], **f64),
            "eval": torch.empty(L["eval_elems"], **f64),
            "evec": torch.empty(L["v_elems"], **f64),
            "t": torch.empty(L["t_doubles"], **f64),
            "delta": torch.empty(L["delta_elems"], **f64),
            "mix": torch.empty(L["mix_elems"], **f64),
            "s_dev": torch.empty(L["delta_elems"], **f64),
            "eig_status": torch.empty(L["n_items"], dtype=torch.int32, device=device),
            "t_status": torch.empty(L["n_items"], dtype=torch.int32, device=device),
        }

    def path_args(self, u, bufs, tlab=None, sigma=None, coef=None):
        """wpcd_path_args over the buffers of alloc() (u, coef: device tensors or None)."""
        import torch
        L = self.layout
        a = _PathArgs()
        if u is not None:
            a.u_fine = _ptr(u, u.dtype, L["u_elems"], "u").value
            a.u_dtype = DTYPE_F32 if u.dtype == torch.float32 else DTYPE_F64
        if coef is not None:
            a.coef = _ptr(coef, torch.float64, L["coef_elems"], "coef").value
        for f, k, dt, n in (("v64", "v64", torch.float64, L["v_elems"]), ("eval", "eval", torch.float64, L["eval_elems"]),
                            ("evec", "evec", torch.float64, L["v_elems"]),
                            ("eig_status", "eig_status", torch.int32, L["n_items"]),
                            ("t", "t", torch.float64, L["t_doubles"]), ("t_status", "t_status", torch.int32, L["n_items"]),
                            ("delta_deg", "delta", torch.float64, L["delta_elems"]),
                            ("mix_deg", "mix", torch.float64, L["mix_elems"]),
                            ("s_dev", "s_dev", torch.float64, L["delta_elems"])):
            setattr(a, f, _ptr(bufs[k], dt, n, k).value)
        if tlab is not None:
            a.n_tlab = tlab.numel()
            a.tlab_mev = _ptr(tlab, torch.float64, a.n_tlab, "tlab").value
            a.sigma_mb = _ptr(sigma, torch.float64, L["n_samples"] * a.n_tlab, "sigma").value
        return a

    def run_path(self, u, bufs, mode, tlab=None, sigma=None, stream=None, coef=None):
        """The whole path in one library call (wpcd_run)."""
        a = self.path_args(u, bufs, tlab, sigma, coef)
        _check(lib().wpcd_run(self._h, ctypes.byref(a), mode, _stream(stream)))

    def graph(self, u, bufs, mode, tlab=None, sigma=None, coef=None) -> "Graph":
        """A HIP graph of the whole path on these buffers (wpcd_graph_create)."""
        a = self.path_args(u, bufs, tlab, sigma, coef)
        h = ctypes.c_void_p()
        _check(lib().wpcd_graph_create(self._h, ctypes.byref(a), mode, ctypes.byref(h)))
        return Graph(h, self)

    def autotune(self, u, bufs, mode, tlab=None, sigma=None, coef=None, reps=2, cache_path=None,
                 stream=None) -> dict:
        """wpcd_autotune: time the candidate schedules on this batch, keep the fastest in the context."""
        a = self.path_args(u, bufs, tlab, sigma, coef)
        r = _TuneResult()
        cp = cache_path.encode() if cache_path else None
        _check(lib().wpcd_autotune(self._h, ctypes.byref(a), mode, reps, cp, ctypes.byref(r), _stream(stream)))
        return {"jacobi_block": r.jacobi_block, "refine_gemm": r.refine_gemm, "from_cache": bool(r.from_cache),
                "best_ms": r.best_ms, "cand_ms": list(r.cand_ms)[:r.n_cand]}

    # ------------------------------------------------------------ steps
    def project(self, u, v64, stream=None):
        import torch
        dt = DTYPE_F32 if u.dtype == torch.float32 else DTYPE_F64
        _check(lib().wpcd_project(self._h, _ptr(u, u.dtype, self.layout["u_elems"], "u"), dt,
                                  _ptr(v64, torch.float64, self.layout["v_elems"], "v64"), _stream(stream)))

    def project_affine(self, coef, v64, stream=None):
        import torch
        L = self.layout
        cp = _ptr(coef, torch.float64, L["coef_elems"], "coef") if coef is not None else ctypes.c_void_p(0)
        _check(lib().wpcd_project_affine(self._h, cp, _ptr(v64, torch.float64, L["v_elems"], "v64"),
                                         _stream(stream)))

    def eigh(self, v64, mode, eval_, evec, status, stream=None, noalloc=False):
        """wpcd_eigh, or wpcd_eigh_noalloc (static device scratch) when noalloc is set."""
        import torch
        L = self.layout
        f = lib().wpcd_eigh_noalloc if noalloc else lib().wpcd_eigh
        _check(f(self._h, _ptr(v64, torch.float64, L["v_elems"], "v64"), mode,
                 _ptr(eval_, torch.float64, L["eval_elems"], "eval"),
                 _ptr(evec, torch.float64, L["v_elems"], "evec"),
                 _ptr(status, torch.int32, L["n_items"], "status"), _stream(stream)))

    def tmatrix(self, v64, eval_, evec, mode, t, status, stream=None):
        import torch
        L = self.layout
        _check(lib().wpcd_tmatrix(self._h, _ptr(v64, torch.float64, L["v_elems"], "v64"),
                                  _ptr(eval_, torch.float64, L["eval_elems"], "eval"),
                                  _ptr(evec, torch.float64, L["v_elems"], "evec"), mode,
                                  _ptr(t, torch.float64, L["t_doubles"], "t"),
                                  _ptr(status, torch.int32, L["n_items"], "status"), _stream(stream)))

    def observables(self, t, delta, mix, s_dev=None, stream=None):
        import torch
        L = self.layout
        sd = _ptr(s_dev, torch.float64, L["delta_elems"], "s_dev") if s_dev is not None else ctypes.c_void_p(0)
        _check(lib().wpcd_observables(self._h, _ptr(t, torch.float64, L["t_doubles"], "t"),
                                      _ptr(delta, torch.float64, L["delta_elems"], "delta"),
                                      _ptr(mix, torch.float64, L["mix_elems"], "mix"), sd, _stream(stream)))

    def sigma_tot(self, delta, mix, tlab, sigma, stream=None):
        import torch
        L = self.layout
        n_tlab = tlab.numel()
        _check(lib().wpcd_sigma_tot(self._h, _ptr(delta, torch.float64, L["delta_elems"], "delta"),
                                    _ptr(mix, torch.float64, L["mix_elems"], "mix"),
                                    _ptr(tlab, torch.float64, n_tlab, "tlab"), n_tlab,
                                    _ptr(sigma, torch.float64, L["n_samples"] * n_tlab, "sigma"),
                                    _stream(stream)))

    def jacobi_launches(self, clear: bool = False) -> dict:
        """Kernel launches and sweeps enqueued by the batch's device-memory Jacobi."""
        c = (ctypes.c_int64 * 2)()
        _check(lib().wpcd_batch_jacobi_launches(self._h, int(bool(clear)), c))
        return {"launches": c[0], "sweeps": c[1]}

    def sigma_band(self, delta, mix, tlab, fracs, sigma_lo, sigma_hi, stream=None):
        """wpcd_sigma_band: lowest and highest sigma_tot over interpolation points."""
        import torch
        L = self.layout
        n_tlab, n_frac = tlab.numel(), fracs.numel()
        _check(lib().wpcd_sigma_band(self._h, _ptr(delta, torch.float64, L["delta_elems"], "delta"),
                                     _ptr(mix, torch.float64, L["mix_elems"], "mix"),
                                     _ptr(tlab, torch.float64, n_tlab, "tlab"), n_tlab,
                                     _ptr(fracs, torch.float64, n_frac, "fracs"), n_frac,
                                     _ptr(sigma_lo, torch.float64, L["n_samples"] * n_tlab, "sigma_lo"),
                                     _ptr(sigma_hi, torch.float64, L["n_samples"] * n_tlab, "sigma_hi"),
                                     _stream(stream)))

    def saclay(self, delta, mix, tlab, theta_deg, amp, dsdo, stream=None):
        """wpcd_saclay: Saclay amplitudes (amp: 10 doubles per sample, energy and
        angle, or None) and dsigma/dOmega (mb/sr) at the T_lab values and c.m.
        angles (degrees) given as device tensors."""
        import torch
        L = self.layout
        nt, nth = tlab.numel(), theta_deg.numel()
        ap = _ptr(amp, torch.float64, L["n_samples"] * nt * nth * 10, "amp") if amp is not None else ctypes.c_void_p(0)
        _check(lib().wpcd_saclay(self._h, _ptr(delta, torch.float64, L["delta_elems"], "delta"),
                                 _ptr(mix, torch.float64, L["mix_elems"], "mix"), _ptr(tlab, torch.float64, nt, "tlab"),
                                 nt, _ptr(theta_deg, torch.float64, nth, "theta"), nth, ap,
                                 _ptr(dsdo, torch.float64, L["n_samples"] * nt * nth, "dsdo"), _stream(stream)))

    def run(self, u, bufs, mode, tlab=None, sigma=None, stream=None, coef=None):
        """The whole path for this batch on one stream: fine-mesh items
        projected from `u`, basis items from `coef`, then eigenpairs, T,
        phase shifts and (with tlab) cross sections."""
        if u is not None:
            self.project(u, bufs["v64"], stream)
        if coef is not None:
            self.project_affine(coef, bufs["v64"], stream)
        self.eigh(bufs["v64"], mode, bufs["eval"], bufs["evec"], bufs["eig_status"], stream)
        self.tmatrix(bufs["v64"], bufs["eval"], bufs["evec"], mode, bufs["t"], bufs["t_status"], stream)
        self.observables(bufs["t"], bufs["delta"], bufs["mix"], bufs["s_dev"], stream)
        if tlab is not None:
            self.sigma_tot(bufs["delta"], bufs["mix"], tlab, sigma, stream)


class Graph:
    """Instantiated HIP graph of a batch's whole path (keeps the batch alive)."""

    def __init__(self, h, batch):
        self._h, self.batch = h, batch
        n = ctypes.c_int64()
        _check(lib().wpcd_graph_nodes(h, ctypes.byref(n)))
        self.nodes = n.value

    def launch(self, stream=None):
        _check(lib().wpcd_graph_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            lib().wpcd_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- matrix inversion
class MiSolver:
    """Batched matrix-inversion (K-matrix) solver: items (n_ch, J, sample_id)
    solved at every T_lab of the list with n_q Gauss nodes on [0, cutoff]."""

    def __init__(self, ctx: Context, items, n_q: int, cutoff: float, tlab):
        arr = (_MiItem * len(items))()
        for i, (n_ch, J, sid) in enumerate(items):
            arr[i] = _MiItem(n_ch, J, sid, 0)
        tl = np.ascontiguousarray(tlab, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().wpcd_mi_create(ctx._h, arr, len(items), n_q, cutoff,
                                    tl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), tl.size, ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.items = list(items)
        self.n_q, self.n_e = n_q, tl.size
        pts, w = np.empty(n_q + tl.size), np.empty(n_q)
        _check(lib().wpcd_mi_points(h, pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self.points, self.weights = pts, w
        lay = _MiLayout()
        offs = [np.zeros(len(items), dtype=np.int64) for _ in range(4)]
        _check(lib().wpcd_mi_layout_get(h, ctypes.byref(lay),
                                        *[o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for o in offs]))
        self.layout = {f: getattr(lay, f) for f, _ in _MiLayout._fields_}
        self.u_off, self.k_off, self.delta_off, self.mix_off = offs

    def close(self):
        if getattr(self, "_h", None):
            lib().wpcd_mi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, device="cuda"):
        import torch
        L = self.layout
        f64 = dict(dtype=torch.float64, device=device)
        return {"kmat": torch.empty(L["kmat_elems"], **f64), "delta": torch.empty(L["delta_elems"], **f64),
                "mix": torch.empty(L["mix_elems"], **f64), "sigma": torch.empty(L["n_samples"] * L["n_e"], **f64),
                "status": torch.empty(L["n_items"], dtype=torch.int32, device=device)}

    def solve(self, u, bufs, stream=None, sigma=True):
        import torch
        L = self.layout
        sg = _ptr(bufs["sigma"], torch.float64, L["n_samples"] * L["n_e"], "sigma") if sigma else ctypes.c_void_p(0)
        _check(lib().wpcd_mi_solve(self._h, _ptr(u, torch.float64, L["u_elems"], "u"),
                                   _ptr(bufs["kmat"], torch.float64, L["kmat_elems"], "kmat"),
                                   _ptr(bufs["delta"], torch.float64, L["delta_elems"], "delta"),
                                   _ptr(bufs["mix"], torch.float64, L["mix_elems"], "mix"), sg,
                                   _ptr(bufs["status"], torch.int32, L["n_items"], "status"), _stream(stream)))


# ---------------------------------------------------------------- serving
class Ticket:
    """A submitted request: its id and the host arrays its results go to."""

    def __init__(self, tid, sigma, delta, mix, status):
        self.id = tid
        self.sigma = sigma
        self.delta = delta
        self.mix = mix
        self.status = status
        self.code = None          # set by Server.poll once done


class Server:
    """Request loop with continuous batching over a context's registered bases."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 4 << 30, max_inflight: int = 4,
                 max_batch_items: int = 4096, max_queue: int = 65536):
        cfg = _ServerConfig(hbm_budget_bytes, max_inflight, max_batch_items, max_queue, 0)
        h = ctypes.c_void_p()
        _check(lib().wpcd_server_create(ctx._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "_h", None):
            lib().wpcd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, channels, tlab, want_phases: bool = False) -> Ticket:
        """channels: list of (basis, J, coefficients); tlab: T_lab values (MeV)."""
        arr = (_ReqChannel * len(channels))()
        keep = []
        n_delta = n_mix = 0
        for i, (basis, J, coef) in enumerate(channels):
            c = np.ascontiguousarray(coef, dtype=np.float64)
            if c.size != basis.n_terms:
                raise ValueError(f"channel {i}: {basis.n_terms} coefficients expected, got {c.size}")
            keep.append(c)
            arr[i] = _ReqChannel(basis.id, J, c.ctypes.data)
            n_delta += basis.grid.n_wp * basis.n_ch
            n_mix += basis.grid.n_wp
        tl = np.ascontiguousarray(tlab, dtype=np.float64)
        sigma = np.full(tl.size, np.nan)
        status = np.zeros(len(channels), dtype=np.int32)
        delta = np.full(n_delta, np.nan) if want_phases else None
        mix = np.full(n_mix, np.nan) if want_phases else None
        req = _Request(arr, len(channels), tl.size, tl.ctypes.data if tl.size else None,
                       sigma.ctypes.data if tl.size else None, delta.ctypes.data if want_phases else None,
                       mix.ctypes.data if want_phases else None, status.ctypes.data)
        t = ctypes.c_uint64()
        _check(lib().wpcd_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return Ticket(t.value, sigma, delta, mix, status)

    def poll(self, ticket: Ticket) -> bool:
        """True once the request is done (ticket.code holds its status)."""
        if ticket.code is not None:
            return True
        code = lib().wpcd_poll(self._h, ticket.id)
        if code == WPCD_ERR_AGAIN:
            return False
        if code == WPCD_ERR_INVALID:
            _check(code)
        ticket.code = code
        return True

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().wpcd_server_stats_get(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}
