"""ctypes binding of libpmx.so (include/pmx.h, include/pmx_probe.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Device buffers are torch tensors on the current device (complex128 for
densities and far fields); the current torch stream is passed to every call.
The library must have been built (``__graft_entry__.build()``); loading fails
loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmx.so")
_lib = None

PMX_STATUS = {0: "PMX_OK", 1: "PMX_EINVAL", 2: "PMX_EGEOM", 3: "PMX_ENOMEM", 4: "PMX_EHIP",
              5: "PMX_ESINGULAR", 6: "PMX_ENOTCONV"}

EXPORTS = [
    "pmx_options_default", "pmx_factor_create", "pmx_solve_plane_waves", "pmx_solve",
    "pmx_far_field", "pmx_factor_info", "pmx_factor_destroy", "pmx_status_string",
    "pmx_last_error", "pmx_probe_bessel", "pmx_probe_diag_block", "pmx_probe_entries",
    "pmx_probe_zgemm", "pmx_probe_lu_solve", "pmx_probe_id", "pmx_plan_query",
    "pmx_probe_cgemm", "pmx_probe_lu_solve_c32", "pmx_probe_id_c32", "pmx_probe_apply",
    "pmx_mlp_opts_default", "pmx_id_dataset", "pmx_mlp_train", "pmx_mlp_predict", "pmx_probe_mlp",
    "pmx_autotune", "pmx_device_cache", "pmx_far_field_noalloc", "pmx_probe_apply_structure",
    "pmx_factor_refactor", "pmx_probe_diag_block_quad", "pmx_plan_members",
]


class PmxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{PMX_STATUS.get(status, status)}: {msg}")
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("m", C.c_int32), ("node_off", C.POINTER(C.c_int64)),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("dx", C.POINTER(C.c_double)), ("dy", C.POINTER(C.c_double)),
                ("ddx", C.POINTER(C.c_double)), ("ddy", C.POINTER(C.c_double)),
                ("center", C.POINTER(C.c_double)), ("grid_ij", C.POINTER(C.c_int32)),
                ("k_ext", C.c_double), ("eps_ext", C.c_double),
                ("k_int", C.POINTER(C.c_double)), ("eps_int", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("id_tol", C.c_double), ("proxy_ratio", C.c_double), ("proxy_min", C.c_int32),
                ("proxy_rule", C.c_int32), ("near_rule", C.c_int32), ("precision", C.c_int32),
                ("timing", C.c_int32), ("ir_max_iter", C.c_int32), ("ir_tol", C.c_double),
                ("solve_graph", C.c_int32), ("learned", C.c_int32), ("model_path", C.c_char_p),
                ("timing_kernels", C.c_uint32), ("reserved0", C.c_int32), ("tune_path", C.c_char_p),
                ("refactor", C.c_int32), ("quadrature", C.c_int32), ("tree", C.c_int32),
                ("leaf_size", C.c_int32), ("eta", C.c_double), ("reserved", C.c_int32 * 2)]


class Info(C.Structure):
    _fields_ = [("levels", C.c_int32), ("root_size", C.c_int32), ("n_unknowns", C.c_int32),
                ("cells", C.c_int32 * 32), ("rank_min", C.c_int32 * 32), ("rank_max", C.c_int32 * 32),
                ("rank_mean", C.c_double * 32), ("bytes_factor", C.c_double),
                ("t_factor_ms", C.c_double), ("t_phase_ms", C.c_double * 16),
                ("t_kernel_ms", C.c_double * 16), ("n_kernel_launch", C.c_int32 * 16),
                ("kernel_bytes", C.c_double * 16), ("kernel_flops", C.c_double * 16),
                ("t_solve_ms", C.c_double), ("ir_iterations", C.c_int32), ("ir_residual", C.c_double),
                ("ir_history", C.c_double * 16), ("id_learned", C.c_int32), ("id_fallback", C.c_int32),
                ("apply_stats", C.c_double * 8), ("factor_launches", C.c_int64),
                ("factor_host_syncs", C.c_int64), ("refactor_launches", C.c_int64),
                ("refactor_graph_nodes", C.c_int64), ("refactor_host_syncs", C.c_int64),
                ("t_refactor_ms", C.c_double)]


class MlpOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("hidden", C.c_int32), ("layers", C.c_int32),
                ("lr", C.c_float), ("wmse", C.c_float), ("seed", C.c_uint64)]

QUADRATURE = {"kress": 0, "zeta": 1}   # self-block rule of pmx_options.quadrature
TREE = {"quad": 0, "kmeans": 1}         # pmx_options.tree

KERNEL_NAMES = ["k_ts_leaf", "k_ts_update", "k_getrf_panel", "k_cpqr_update", "k_cpqr", "k_zgemm",
                "k_trsm_small", "k_entries", "k_diag_pairs/maue", "k_apply_off", "k_getrs_small"]


def _check_one_hip_runtime():
    """Exactly one HIP runtime may be mapped into the process: a second copy next to
    torch's (the library bound to another libamdhip64) gives device pointers that one of
    them does not know, and the first GPU call crashes."""
    try:
        maps = open("/proc/self/maps").read().splitlines()
    except OSError:
        return
    paths = {os.path.realpath(l.split()[-1]) for l in maps if "libamdhip64.so" in l and "/" in l}
    if len(paths) > 1:
        raise RuntimeError("two HIP runtimes are loaded (" + ", ".join(sorted(paths)) + "); libpmx.so must bind "
                           "to the one torch loaded")


def load(path=None):
    """Load libpmx.so (once)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    # PyTorch bundles its own HIP runtime under the same soname; importing it first makes
    # the library bind to that one runtime instead of loading a second copy.
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise RuntimeError(f"libpmx.so is not built ({p}); run __graft_entry__.build()")
    lib = C.CDLL(p)
    _check_one_hip_runtime()
    vp = C.c_void_p
    lib.pmx_options_default.argtypes = [C.POINTER(Options)]
    lib.pmx_options_default.restype = None
    lib.pmx_factor_create.argtypes = [C.POINTER(Geometry), C.POINTER(Options), vp, C.POINTER(vp)]
    lib.pmx_solve_plane_waves.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), vp, vp]
    lib.pmx_solve.argtypes = [vp, C.c_int32, vp, vp, vp]
    lib.pmx_far_field.argtypes = [vp, C.c_int32, vp, C.c_int32, C.POINTER(C.c_double), vp, vp]
    lib.pmx_far_field_noalloc.argtypes = [vp, C.c_int32, vp, C.c_int32, C.POINTER(C.c_double), vp, vp]
    lib.pmx_factor_info.argtypes = [vp, C.POINTER(Info)]
    lib.pmx_factor_destroy.argtypes = [vp]
    lib.pmx_factor_destroy.restype = None
    lib.pmx_status_string.argtypes = [C.c_int]
    lib.pmx_status_string.restype = C.c_char_p
    lib.pmx_last_error.argtypes = []
    lib.pmx_last_error.restype = C.c_char_p
    lib.pmx_probe_bessel.argtypes = [vp, C.c_int64, vp, vp]
    lib.pmx_probe_diag_block.argtypes = [C.POINTER(Geometry), C.c_int32, vp, vp]
    lib.pmx_probe_diag_block_quad.argtypes = [C.POINTER(Geometry), C.c_int32, C.c_int32, vp, vp]
    ip = C.POINTER(C.c_int32)
    lib.pmx_probe_entries.argtypes = [C.POINTER(Geometry), C.c_int32, ip, ip, C.c_int32, ip, ip, vp, vp]
    lib.pmx_probe_zgemm.argtypes = [C.c_int32] * 6 + [vp, vp, vp, vp]
    lib.pmx_probe_lu_solve.argtypes = [C.c_int32, C.c_int32, vp, vp, C.c_int32, vp, ip, C.c_int32, vp]
    lib.pmx_probe_id.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, C.c_double, ip, vp, ip, vp, vp]
    lib.pmx_probe_cgemm.argtypes = [C.c_int32] * 6 + [vp, vp, vp, vp]
    lib.pmx_probe_lu_solve_c32.argtypes = [C.c_int32, C.c_int32, vp, vp, C.c_int32, vp, ip, C.c_int32, vp]
    lib.pmx_probe_id_c32.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, C.c_double, ip, vp, ip, vp, vp]
    lib.pmx_probe_apply.argtypes = [C.POINTER(Geometry), C.c_int32, vp, vp, vp]
    lib.pmx_probe_apply_structure.argtypes = [C.POINTER(Geometry), C.POINTER(Options), C.c_int32,
                                              C.POINTER(C.c_double)]
    fp = C.POINTER(C.c_float)
    lib.pmx_mlp_opts_default.argtypes = [C.POINTER(MlpOpts)]
    lib.pmx_mlp_opts_default.restype = None
    lib.pmx_id_dataset.argtypes = [C.POINTER(Geometry), C.POINTER(Options), C.c_char_p, C.c_int32, vp]
    lib.pmx_mlp_train.argtypes = [C.c_char_p, C.POINTER(MlpOpts), C.c_char_p, C.POINTER(C.c_double), vp]
    lib.pmx_mlp_predict.argtypes = [C.c_char_p, C.POINTER(Geometry), C.POINTER(Options), fp, vp]
    lib.pmx_probe_mlp.argtypes = [C.c_int32] * 4 + [fp, fp, fp, C.c_int32, C.c_float, fp, fp,
                                                    C.POINTER(C.c_double), vp]
    lib.pmx_autotune.argtypes = [C.POINTER(Geometry), C.POINTER(Options), C.c_int32, C.c_int32, C.c_char_p, vp]
    lib.pmx_device_cache.argtypes = [C.c_int64, C.POINTER(C.c_int64)]
    dp = C.POINTER(C.c_double)
    lib.pmx_plan_query.argtypes = [C.POINTER(Geometry), C.POINTER(Options), C.c_int32, C.c_int32,
                                   ip, ip, ip, ip, ip, dp, dp, dp, ip, ip, ip]
    lib.pmx_plan_members.argtypes = [C.POINTER(Geometry), C.POINTER(Options), C.c_int32, C.c_int32, C.c_int32,
                                     ip, ip, ip, ip, ip, ip, ip]
    for name in EXPORTS:
        if name not in ("pmx_options_default", "pmx_factor_destroy", "pmx_status_string",
                        "pmx_last_error", "pmx_mlp_opts_default"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(st):
    if st != 0:
        raise PmxError(st, _lib.pmx_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _GeomKeep:
    """Host arrays of a workload kept alive while a Geometry structure points at them."""

    def __init__(self, w, eps_int=None):
        self.node_off = np.ascontiguousarray(w.node_off, dtype=np.int64)
        self.arr = [np.ascontiguousarray(a, dtype=np.float64) for a in (w.x, w.y, w.dx, w.dy, w.ddx, w.ddy)]
        self.center = np.ascontiguousarray(np.asarray(w.centers, float).reshape(-1))
        gi = w.grid_index if w.grid_index is not None else np.zeros((w.m, 2), int)
        self.grid = np.ascontiguousarray(np.asarray(gi).reshape(-1), dtype=np.int32)
        self.k_int = np.ascontiguousarray(w.k_int, dtype=np.float64)
        self.eps_int = None if eps_int is None else np.ascontiguousarray(eps_int, dtype=np.float64)
        g = Geometry()
        g.m = w.m
        g.node_off = _ptr(self.node_off, C.c_int64)
        g.x, g.y, g.dx, g.dy, g.ddx, g.ddy = [_ptr(a, C.c_double) for a in self.arr]
        g.center = _ptr(self.center, C.c_double)
        g.grid_ij = _ptr(self.grid, C.c_int32) if w.grid_index is not None else None
        g.k_ext = w.k_ext
        g.eps_ext = w.eps_ext
        g.k_int = _ptr(self.k_int, C.c_double)
        g.eps_int = None if self.eps_int is None else _ptr(self.eps_int, C.c_double)
        self.g = g


def options(w=None, **kw):
    """Solver options: the library's defaults, the workload's plan settings, then kw.  A
    model_path string is kept alive by the returned structure's _keep attribute."""
    load()
    o = Options()
    _lib.pmx_options_default(C.byref(o))
    if w is not None:
        o.id_tol = w.id_tol
        o.proxy_ratio = w.proxy_ratio
        o.proxy_min = w.proxy_min
        o.proxy_rule = 0 if w.proxy_paper_rule else 1
        o.near_rule = w.near_rule
        o.quadrature = QUADRATURE[getattr(w, "quadrature", "kress")]
        o.tree = TREE[getattr(w, "tree", "quad")]
        o.leaf_size = int(getattr(w, "leaf_size", 4))
        o.eta = float(getattr(w, "eta", 1.0))
    keep = []
    for k, v in kw.items():
        if k in ("model_path", "tune_path") and isinstance(v, str):
            v = v.encode()
            keep.append(v)
        setattr(o, k, v)
    o._keep = keep
    return o


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Factor:
    """A factorisation held by the library; `solve_plane_waves` returns torch tensors."""

    def __init__(self, w, opts=None):
        load()
        self.w = w
        self._keep = _GeomKeep(w)
        self.opts = options(w) if opts is None else opts
        h = C.c_void_p()
        _check(_lib.pmx_factor_create(C.byref(self._keep.g), C.byref(self.opts), _stream(), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.pmx_factor_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = Info()
        _check(_lib.pmx_factor_info(self.h, C.byref(i)))
        return i

    def refactor(self, k_int, eps_int=None):
        """pmx_factor_refactor: the kept numeric phase replayed for new interior media
        (k_int per inclusion, eps_int per inclusion or None)."""
        k = np.ascontiguousarray(k_int, dtype=np.float64)
        if k.shape != (self.w.m,):
            raise ValueError("k_int needs one value per inclusion")
        e = None if eps_int is None else np.ascontiguousarray(eps_int, dtype=np.float64)
        if e is not None and e.shape != (self.w.m,):
            raise ValueError("eps_int needs one value per inclusion")
        _check(_lib.pmx_factor_refactor(self.h, _ptr(k, C.c_double), None if e is None else _ptr(e, C.c_double),
                                        _stream()))

    def solve_plane_waves(self, angles, out=None):
        import torch
        ang = np.ascontiguousarray(angles, dtype=np.float64)
        n2 = self.w.n_unknowns
        if out is None:
            out = torch.empty((len(ang), n2), dtype=torch.complex128, device="cuda")
        _check(_lib.pmx_solve_plane_waves(self.h, len(ang), _ptr(ang, C.c_double), C.c_void_p(out.data_ptr()),
                                          _stream()))
        return out

    def solve(self, rhs, out=None):
        import torch
        rhs = rhs.contiguous()
        if out is None:
            out = torch.empty_like(rhs)
        _check(_lib.pmx_solve(self.h, rhs.shape[0], C.c_void_p(rhs.data_ptr()), C.c_void_p(out.data_ptr()),
                              _stream()))
        return out

    def far_field(self, dens, dirs):
        import torch
        d = np.ascontiguousarray(dirs, dtype=np.float64)
        dens = dens.contiguous()
        out = torch.empty((dens.shape[0], len(d)), dtype=torch.complex128, device=dens.device)
        _check(_lib.pmx_far_field(self.h, dens.shape[0], C.c_void_p(dens.data_ptr()), len(d), _ptr(d, C.c_double),
                                  C.c_void_p(out.data_ptr()), _stream()))
        return out

    def far_field_noalloc(self, dens, dirs, out=None):
        """pmx_far_field_noalloc: the same pattern with the partial sums in the library's
        static per-GPU array (no device allocation; `out` may be given)."""
        import torch
        d = np.ascontiguousarray(dirs, dtype=np.float64)
        dens = dens.contiguous()
        if out is None:
            out = torch.empty((dens.shape[0], len(d)), dtype=torch.complex128, device=dens.device)
        _check(_lib.pmx_far_field_noalloc(self.h, dens.shape[0], C.c_void_p(dens.data_ptr()), len(d),
                                          _ptr(d, C.c_double), C.c_void_p(out.data_ptr()), _stream()))
        return out


def dens_to_numpy(d, w):
    """(nrhs, 2N) tensor -> (2N, nrhs) numpy, the oracle's stacked layout."""
    return d.detach().cpu().numpy().T.copy()


# -- probes -------------------------------------------------------------------------
def probe_bessel(z):
    import torch
    load()
    zt = torch.as_tensor(np.ascontiguousarray(z, dtype=np.float64), device="cuda")
    out = torch.empty((4, len(z)), dtype=torch.float64, device="cuda")
    _check(_lib.pmx_probe_bessel(C.c_void_p(zt.data_ptr()), len(z), C.c_void_p(out.data_ptr()), _stream()))
    return out.cpu().numpy()


def probe_diag_block(w, j):
    """The self block of inclusion j by the workload's quadrature (w.quadrature)."""
    import torch
    load()
    keep = _GeomKeep(w)
    n = int(w.node_off[j + 1] - w.node_off[j])
    out = torch.empty((2 * n, 2 * n), dtype=torch.complex128, device="cuda")
    _check(_lib.pmx_probe_diag_block_quad(C.byref(keep.g), j, QUADRATURE[getattr(w, "quadrature", "kress")],
                                          C.c_void_p(out.data_ptr()), _stream()))
    return out.cpu().numpy().T.copy()       # column major on the device


def probe_entries(w, rows, rtyp, cols, ctyp):
    import torch
    load()
    keep = _GeomKeep(w)
    r = np.ascontiguousarray(rows, np.int32)
    rt = np.ascontiguousarray(rtyp, np.int32)
    c = np.ascontiguousarray(cols, np.int32)
    ct = np.ascontiguousarray(ctyp, np.int32)
    out = torch.empty((len(c), len(r)), dtype=torch.complex128, device="cuda")
    _check(_lib.pmx_probe_entries(C.byref(keep.g), len(r), _ptr(r, C.c_int32), _ptr(rt, C.c_int32), len(c),
                                  _ptr(c, C.c_int32), _ptr(ct, C.c_int32), C.c_void_p(out.data_ptr()), _stream()))
    return out.cpu().numpy().T.copy()


def _colmajor(t):
    """(batch, rows, cols) torch -> device buffer holding each matrix column major."""
    return t.transpose(-1, -2).contiguous()


def _ctype(fp32):
    import torch
    return torch.complex64 if fp32 else torch.complex128


def probe_zgemm(A, B, opa=0, opb=0, fp32=False):
    """A, B: (batch, ., .) complex numpy arrays in their stored shapes; fp32 runs the
    complex FP32 kernel on the inputs rounded to complex64."""
    import torch
    load()
    ct = _ctype(fp32)
    At = _colmajor(torch.as_tensor(A, device="cuda").to(ct))
    Bt = _colmajor(torch.as_tensor(B, device="cuda").to(ct))
    batch = A.shape[0]
    m = A.shape[1] if opa == 0 else A.shape[2]
    k = A.shape[2] if opa == 0 else A.shape[1]
    n = B.shape[2] if opb == 0 else B.shape[1]
    Ct = torch.empty((batch, n, m), dtype=ct, device="cuda")
    fn = _lib.pmx_probe_cgemm if fp32 else _lib.pmx_probe_zgemm
    _check(fn(batch, m, n, k, opa, opb, C.c_void_p(At.data_ptr()), C.c_void_p(Bt.data_ptr()),
              C.c_void_p(Ct.data_ptr()), _stream()))
    return Ct.transpose(-1, -2).cpu().numpy()


def probe_lu_solve(A, B, fp32=False, variant=-1):
    import torch
    load()
    ct = _ctype(fp32)
    batch, n, _ = A.shape
    nrhs = B.shape[2]
    At = _colmajor(torch.as_tensor(A, device="cuda").to(ct))
    Bt = _colmajor(torch.as_tensor(B, device="cuda").to(ct))
    piv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = np.zeros(batch, np.int32)
    fn = _lib.pmx_probe_lu_solve_c32 if fp32 else _lib.pmx_probe_lu_solve
    _check(fn(batch, n, C.c_void_p(At.data_ptr()), C.c_void_p(piv.data_ptr()), nrhs,
              C.c_void_p(Bt.data_ptr()), _ptr(info, C.c_int32), int(variant), _stream()))
    return (At.transpose(-1, -2).cpu().numpy(), piv.cpu().numpy(), Bt.transpose(-1, -2).cpu().numpy(), info)


def probe_id(M, tol, kmin=None, fp32=False):
    import torch
    load()
    ct = _ctype(fp32)
    batch, m, c = M.shape
    Mt = _colmajor(torch.as_tensor(M, device="cuda").to(ct))
    piv = torch.empty((batch, c), dtype=torch.int32, device="cuda")
    rank = np.zeros(batch, np.int32)
    T = torch.zeros((batch, c, c), dtype=ct, device="cuda")
    km = None if kmin is None else np.ascontiguousarray(kmin, np.int32)
    fn = _lib.pmx_probe_id_c32 if fp32 else _lib.pmx_probe_id
    _check(fn(batch, m, c, C.c_void_p(Mt.data_ptr()), tol, None if km is None else _ptr(km, C.c_int32),
              C.c_void_p(piv.data_ptr()), _ptr(rank, C.c_int32), C.c_void_p(T.data_ptr()), _stream()))
    return piv.cpu().numpy(), rank, T.transpose(-1, -2).cpu().numpy()


def probe_apply(w, x):
    """y = A x with the library's dense FP64 operator; x numpy (2N, nrhs) in the oracle's
    stacked layout, returned in the same layout."""
    import torch
    load()
    keep = _GeomKeep(w)
    xt = torch.as_tensor(np.ascontiguousarray(np.asarray(x).T), device="cuda").to(torch.complex128).contiguous()
    y = torch.empty_like(xt)
    _check(_lib.pmx_probe_apply(C.byref(keep.g), xt.shape[0], C.c_void_p(xt.data_ptr()), C.c_void_p(y.data_ptr()),
                                _stream()))
    return y.cpu().numpy().T.copy()


APPLY_STRUCTURE_KEYS = ("m2l_pairs", "mean_source_order", "mean_local_order", "local_expansions", "l2l_pairs",
                        "near_node_pairs", "direct_far_pairs", "table_bytes", "max_m2l_list", "mean_m2l_list",
                        "max_far_list", "max_near_list", "coverage_violations", "waves", "max_local_order",
                        "pairs_checked")


def apply_structure(w, check=False, opts=None):
    """Host-only structure of the refinement's operator apply for workload w (no GPU)."""
    load()
    keep = _GeomKeep(w)
    o = options(w) if opts is None else opts
    st = (C.c_double * 16)()
    _check(_lib.pmx_probe_apply_structure(C.byref(keep.g), C.byref(o), int(bool(check)), st))
    return dict(zip(APPLY_STRUCTURE_KEYS, [float(v) for v in st]))


def plan_query(w, opts=None):
    """Host-only plan of the library: list of levels, each a list of dicts."""
    load()
    keep = _GeomKeep(w)
    o = options(w) if opts is None else opts
    nl, nct, nnt = C.c_int32(), C.c_int32(), C.c_int32()
    z = C.POINTER(C.c_int32)()
    zd_ = C.POINTER(C.c_double)()
    _check(_lib.pmx_plan_query(C.byref(keep.g), C.byref(o), 0, 0, C.byref(nl), C.byref(nct), C.byref(nnt),
                               z, z, zd_, zd_, zd_, z, z, z))
    nc, nn = nct.value, nnt.value
    lev = np.zeros(nc, np.int32)
    first = np.zeros(nc, np.int32)
    cen = np.zeros(2 * nc)
    rc = np.zeros(nc)
    rp = np.zeros(nc)
    P = np.zeros(nc, np.int32)
    noff = np.zeros(nc + 1, np.int32)
    near = np.zeros(max(nn, 1), np.int32)
    _check(_lib.pmx_plan_query(C.byref(keep.g), C.byref(o), nc, nn, C.byref(nl), C.byref(nct), C.byref(nnt),
                               _ptr(lev, C.c_int32), _ptr(first, C.c_int32), _ptr(cen, C.c_double),
                               _ptr(rc, C.c_double), _ptr(rp, C.c_double), _ptr(P, C.c_int32),
                               _ptr(noff, C.c_int32), _ptr(near, C.c_int32)))
    # membership: inclusions and children per cell (same cell order)
    ncm, nit, nkt = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.pmx_plan_members(C.byref(keep.g), C.byref(o), 0, 0, 0, C.byref(ncm), C.byref(nit), C.byref(nkt),
                                 z, z, z, z))
    ioff = np.zeros(nc + 1, np.int32)
    inc = np.zeros(max(nit.value, 1), np.int32)
    koff = np.zeros(nc + 1, np.int32)
    kid = np.zeros(max(nkt.value, 1), np.int32)
    _check(_lib.pmx_plan_members(C.byref(keep.g), C.byref(o), nc, nit.value, nkt.value, C.byref(ncm), C.byref(nit),
                                 C.byref(nkt), _ptr(ioff, C.c_int32), _ptr(inc, C.c_int32), _ptr(koff, C.c_int32),
                                 _ptr(kid, C.c_int32)))
    levels = [[] for _ in range(nl.value)]
    for t in range(nc):
        levels[lev[t]].append(dict(first=int(first[t]), center=(cen[2 * t], cen[2 * t + 1]), rc=rc[t],
                                   Rp=rp[t], P=int(P[t]), near=list(near[noff[t]:noff[t + 1]]),
                                   incl=[int(v) for v in inc[ioff[t]:ioff[t + 1]]],
                                   children=[int(v) for v in kid[koff[t]:koff[t + 1]]]))
    return levels


# -- learned skeleton proposals -------------------------------------------------------
NFEAT = 20
NOUT = 8


def mlp_opts(**kw):
    load()
    o = MlpOpts()
    _lib.pmx_mlp_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def id_dataset(w, path, append=False, opts=None):
    """Full leaf IDs of workload w -> training samples (one per leaf node) in file `path`."""
    load()
    keep = _GeomKeep(w)
    o = options(w) if opts is None else opts
    _check(_lib.pmx_id_dataset(C.byref(keep.g), C.byref(o), str(path).encode(), int(bool(append)), _stream()))


def device_cache(limit=-1):
    """Bytes of device blocks the library keeps from destroyed factors for later ones; a
    limit >= 0 first sets the cache limit and frees what exceeds it (0 empties it)."""
    load()
    held = C.c_int64(0)
    _check(_lib.pmx_device_cache(int(limit), C.byref(held)))
    return held.value


def autotune(w, path, nrhs=None, reps=3, **kw):
    """Launch-parameter table for workload w (options as options(w, **kw)) written to
    `path`; factors take it through options(..., tune_path=path)."""
    load()
    keep = _GeomKeep(w)
    o = options(w, **kw)
    n = len(w.angles) if nrhs is None else int(nrhs)
    _check(_lib.pmx_autotune(C.byref(keep.g), C.byref(o), n, int(reps), str(path).encode(), _stream()))


def read_tune_table(path):
    """{(knob, real_bytes, a, b, c): choice} of a launch-parameter table."""
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if len(line) == 6:
            out[(line[0],) + tuple(int(v) for v in line[1:5])] = int(line[5])
    return out


def read_dataset(path):
    """(X [n, 20], Y [n, 8]) of a training file (float32)."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"PMXIDS01"
    nin, nout = np.frombuffer(raw[8:16], np.int32)
    n = int(np.frombuffer(raw[16:24], np.int64)[0])
    rows = np.frombuffer(raw[24:24 + 4 * n * (nin + nout)], np.float32).reshape(n, nin + nout)
    return rows[:, :nin].copy(), rows[:, nin:].copy()


def mlp_train(data_path, model_path, **kw):
    """Train the proposal network on the device; returns the last epoch's mean loss."""
    load()
    o = mlp_opts(**kw)
    loss = C.c_double()
    _check(_lib.pmx_mlp_train(str(data_path).encode(), C.byref(o), str(model_path).encode(), C.byref(loss),
                              _stream()))
    return loss.value


def mlp_predict(model_path, w, opts=None):
    """The network's outputs per boundary node of w: (n_nodes, 8) float32."""
    load()
    keep = _GeomKeep(w)
    o = options(w) if opts is None else opts
    out = np.zeros((int(w.node_off[-1]), NOUT), np.float32)
    _check(_lib.pmx_mlp_predict(str(model_path).encode(), C.byref(keep.g), C.byref(o), _ptr(out, C.c_float),
                                _stream()))
    return out


def probe_mlp(shape, params, X, labels, wmse=10.0):
    """Forward + backward of the network on host arrays: shape (nin, nhidden, nlayer, nout),
    params packed per layer (W out x in column major, then b), X (B, nin), labels (B, nout).
    Returns (out (B, nout), grad (like params), loss)."""
    load()
    nin, nh, nl, nout = shape
    p = np.ascontiguousarray(params, np.float32)
    x = np.ascontiguousarray(X, np.float32)
    y = np.ascontiguousarray(labels, np.float32)
    B = x.shape[0]
    out = np.zeros((B, nout), np.float32)
    grad = np.zeros_like(p)
    loss = C.c_double()
    _check(_lib.pmx_probe_mlp(nin, nh, nl, nout, _ptr(p, C.c_float), _ptr(x, C.c_float), _ptr(y, C.c_float), B,
                              wmse, _ptr(out, C.c_float), _ptr(grad, C.c_float), C.byref(loss), _stream()))
    return out, grad, loss.value
