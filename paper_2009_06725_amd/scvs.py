"""ctypes binding of libscvs (the gfx950 HIP library declared in include/scvs.h).

Argument marshalling only: every computation runs in the library's kernels.
PyTorch provides device memory (complex128 / float64 / int tensors on a HIP
device) and the stream the library launches on. If the built library is
missing this module raises on import instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscvs.so")

BC_FREE, BC_WALL, BC_DIRICHLET, BC_TRACTION = 0, 1, 2, 3
(X_EDGES, X_C2N, X_ROWPTR, X_COL, X_KS, X_M, X_G, X_MP, X_DIRNODES, X_DMASK, X_LOADS, X_NODEXYZ, X_C21PTR,
 X_C21COL) = range(14)

EXPORTED = [
    "scvs_last_error", "scvs_version", "scvs_ctx_create", "scvs_ctx_destroy", "scvs_ctx_set_mem_cap",
    "scvs_mesh_create",
    "scvs_mesh_destroy", "scvs_mesh_info", "scvs_mesh_set_midside", "scvs_mesh_set_bc", "scvs_mesh_set_windkessel",
    "scvs_assemble",
    "scvs_mesh_export", "scvs_spmv", "scvs_rhs", "scvs_solve_opts_default", "scvs_solve",
    "scvs_autotune", "scvs_solve_groups", "scvs_boundary_norms", "scvs_mode_norms", "scvs_select_modes",
    "scvs_mode_increments", "scvs_mode_norms_noalloc", "scvs_mesh_mg_info", "scvs_synthesize", "scvs_probe_mfma", "scvs_profile_enable", "scvs_profile_read",
    "scvs_ws_create", "scvs_ws_train", "scvs_ws_predict", "scvs_ws_refine", "scvs_ws_destroy", "scvs_ws_export",
    "scvs_ws_set_params", "scvs_ws_loss_grad", "scvs_herm_eig", "scvs_probe_mfma_bf16",
]
WS_SIGMA, WS_BASIS, WS_PARAMS, WS_TARGETS, WS_NPARAM, WS_TMEAN, WS_TSCALE = range(7)


class ScvsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"scvs error {code}: {msg}")
        self.code = code


class MeshInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nv", C.c_int64), ("nc", C.c_int64), ("nf", C.c_int64),
                ("ne", C.c_int64), ("n2", C.c_int64), ("ndof", C.c_int64), ("nnz_s2", C.c_int64),
                ("nnz_c21", C.c_int64), ("ndir", C.c_int64), ("ntraction", C.c_int32),
                ("assembled", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32),
                ("cheb_vel", C.c_int32), ("cheb_pres", C.c_int32), ("cheb_ratio", C.c_double),
                ("max_batch", C.c_int32), ("use_graph", C.c_int32), ("verbose", C.c_int32),
                ("precision", C.c_int32), ("orth", C.c_int32), ("cheb_ratio_pres", C.c_double), ("penalty", C.c_double),
                ("inner_rtol", C.c_double), ("vel_block", C.c_int32), ("pres_block", C.c_int32),
                ("mg_smooth", C.c_int32), ("mg_ratio", C.c_double), ("steady_schur_omega", C.c_double),
                ("mg_post0", C.c_int32)]


class SolveGroup(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("nsys", C.c_int64), ("omega", C.c_void_p), ("traction", C.c_void_p),
                ("g", C.c_void_p), ("x0", C.c_void_p), ("u_out", C.c_void_p), ("p_out", C.c_void_p),
                ("opts", C.c_void_p), ("rep", C.c_void_p)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("bytes", C.c_double)]


class Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
                ("rel_residual", C.c_double), ("warm", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2009_06725_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)
        L.scvs_last_error.restype = C.c_char_p
        L.scvs_version.restype = C.c_char_p
        L.scvs_ctx_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
        L.scvs_ctx_destroy.argtypes = [vp]
        L.scvs_ctx_set_mem_cap.argtypes = [vp, C.c_uint64]
        L.scvs_mesh_create.argtypes = [vp, C.c_int, i64, vp, i64, vp, i64, vp, vp, C.POINTER(vp)]
        L.scvs_mesh_destroy.argtypes = [vp]
        L.scvs_mesh_info.argtypes = [vp, C.POINTER(MeshInfo)]
        L.scvs_mesh_set_midside.argtypes = [vp, i64, vp, vp]
        L.scvs_mesh_set_bc.argtypes = [vp, C.c_int, vp, vp]
        L.scvs_mesh_set_windkessel.argtypes = [vp, C.c_int, vp, vp, vp, vp]
        L.scvs_assemble.argtypes = [vp, C.c_double, C.c_double]
        L.scvs_mesh_export.argtypes = [vp, C.c_int, vp]
        L.scvs_spmv.argtypes = [vp, i64, vp, vp, vp]
        L.scvs_rhs.argtypes = [vp, i64, vp, vp, vp, vp]
        L.scvs_solve_opts_default.argtypes = [C.POINTER(SolveOpts)]
        L.scvs_solve_opts_default.restype = None
        L.scvs_solve.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(Report)]
        L.scvs_autotune.argtypes = [vp, i64, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveOpts),
                                    C.POINTER(C.c_double)]
        L.scvs_solve_groups.argtypes = [C.c_int, vp]
        L.scvs_boundary_norms.argtypes = [vp, i64, vp, vp, vp, vp]
        L.scvs_mode_norms.argtypes = [vp, i64, vp, vp, vp, vp]
        L.scvs_mode_norms_noalloc.argtypes = [vp, i64, vp, vp, vp, vp]
        L.scvs_mesh_mg_info.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, C.POINTER(C.c_int)]
        L.scvs_select_modes.argtypes = [i64, vp, vp, vp, C.c_double, C.c_int, vp, vp, vp]
        L.scvs_mode_increments.argtypes = [i64, vp, vp, vp]
        L.scvs_synthesize.argtypes = [vp, i64, vp, vp, i64, i64, vp, vp]
        L.scvs_probe_mfma.argtypes = [vp, vp, vp, vp]
        L.scvs_profile_enable.argtypes = [vp, C.c_int]
        L.scvs_ws_create.argtypes = [vp, i64, vp, vp, C.c_int, C.c_int, C.c_int, C.c_uint64, C.POINTER(vp)]
        L.scvs_ws_train.argtypes = [vp, C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.scvs_ws_predict.argtypes = [vp, i64, vp, vp, vp]
        L.scvs_ws_refine.argtypes = [vp, i64, vp, vp, vp, vp]
        L.scvs_ws_destroy.argtypes = [vp]
        L.scvs_ws_export.argtypes = [vp, C.c_int, vp]
        L.scvs_ws_set_params.argtypes = [vp, vp]
        L.scvs_ws_loss_grad.argtypes = [vp, i64, vp, vp, C.POINTER(C.c_double), vp]
        L.scvs_herm_eig.argtypes = [C.c_int, vp, vp, vp]
        L.scvs_probe_mfma_bf16.argtypes = [vp, vp, vp, vp]
        L.scvs_profile_read.argtypes = [vp, C.c_int, C.POINTER(KernelStat), C.POINTER(C.c_int)]
        for name in EXPORTED:
            if name not in ("scvs_last_error", "scvs_version", "scvs_solve_opts_default"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise ScvsError(code, lib().scvs_last_error().decode())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


E_INVALID = -1
E_NOMEM = -3
SCVS_NOALLOC_MAX_SYSTEMS = 256  # include/scvs.h


def _dev(t, dtype_name: str, numel: int | None = None, device: int | None = None, what: str = "tensor"):
    """Device pointer of a contiguous torch tensor of the expected dtype, holding
    exactly `numel` elements (when given) on HIP device `device` (when given).
    The C ABI carries no buffer sizes, so these checks are what keeps a kernel
    from reading or writing past a caller's buffer."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise ScvsError(E_INVALID, f"{what}: expected a device tensor")
    if not t.is_contiguous():
        raise ScvsError(E_INVALID, f"{what}: expected a contiguous tensor")
    if str(t.dtype) != dtype_name:
        raise ScvsError(E_INVALID, f"{what}: expected {dtype_name}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ScvsError(E_INVALID, f"{what}: expected {numel} elements, got {t.numel()}")
    if device is not None and t.device.index != device:
        raise ScvsError(E_INVALID, f"{what}: tensor is on device {t.device.index}, the context on {device}")
    return C.c_void_p(t.data_ptr())


def _traction(i, ns: int, traction):
    """Host c128 [ns][ntraction] traction coefficients of ns systems."""
    tr = np.asarray(traction, np.complex128)
    if tr.size != ns * i.ntraction:
        raise ScvsError(E_INVALID, f"traction: expected {ns}x{i.ntraction} values, got {tr.size}")
    return _host(tr.reshape(ns, i.ntraction).view(np.float64) if tr.size else np.zeros(1), np.float64)


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().scvs_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = C.c_void_p()
        _check(lib().scvs_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def set_mem_cap(self, nbytes: int):
        """Device bytes a solve's Krylov slot pool may take (0: 90% of free memory)."""
        _check(lib().scvs_ctx_set_mem_cap(self.h, int(nbytes)))

    def profile(self, on: bool):
        """Time every library kernel launch with HIP events on this context's stream."""
        _check(lib().scvs_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel class: (launches, total_ms, algorithmic bytes)} since the last read."""
        buf = (KernelStat * 64)()
        n = C.c_int()
        _check(lib().scvs_profile_read(self.h, 64, buf, C.byref(n)))
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms, buf[i].bytes) for i in range(n.value)}

    def close(self):
        if self.h:
            _check(lib().scvs_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """A simplex mesh on the device with its quadratic numbering and patterns."""

    def __init__(self, ctx: Context, dim: int, xyz, cells, bfaces, btags):
        self.ctx = ctx
        xyz, px = _host(xyz, np.float64)
        cells, pc = _host(cells, np.int32)
        bfaces, pf = _host(bfaces, np.int32)
        btags, pt = _host(btags, np.int32)
        h = C.c_void_p()
        _check(lib().scvs_mesh_create(ctx.h, dim, xyz.shape[0], px, cells.shape[0], pc,
                                      bfaces.shape[0], pf, pt, C.byref(h)))
        self.h = h

    @classmethod
    def from_workload(cls, ctx: Context, mesh) -> "Mesh":
        m = cls(ctx, mesh.dim, mesh.xyz, mesh.cells, mesh.bfaces, mesh.btags)
        if mesh.curved_edges.shape[0]:
            m.set_midside(mesh.curved_edges, mesh.curved_xyz)
        return m

    def close(self):
        if getattr(self, "h", None):
            _check(lib().scvs_mesh_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> MeshInfo:
        i = MeshInfo()
        _check(lib().scvs_mesh_info(self.h, C.byref(i)))
        return i

    def set_midside(self, edge_vertices, xyz):
        ev, pe = _host(edge_vertices, np.int32)
        x, px = _host(xyz, np.float64)
        _check(lib().scvs_mesh_set_midside(self.h, ev.shape[0], pe, px))

    def set_bc(self, bc: dict):
        tags, pt = _host(list(bc.keys()), np.int32)
        kinds, pk = _host(list(bc.values()), np.int32)
        _check(lib().scvs_mesh_set_bc(self.h, tags.size, pt, pk))

    def set_windkessel(self, outlets: dict):
        """Lumped outlets {traction tag: (rp, c, rd)}; an empty dict removes them."""
        tags, pt = _host(list(outlets.keys()), np.int32)
        prm = np.array(list(outlets.values()), np.float64).reshape(-1, 3)
        rp, pr = _host(prm[:, 0], np.float64)
        cc, pc = _host(prm[:, 1], np.float64)
        rd, pd = _host(prm[:, 2], np.float64)
        _check(lib().scvs_mesh_set_windkessel(self.h, tags.size, pt, pr, pc, pd))

    def assemble(self, rho: float, mu: float):
        _check(lib().scvs_assemble(self.h, rho, mu))

    def export(self, which: int) -> np.ndarray:
        i = self.info
        d = i.dim
        nn = (d + 1) * (d + 2) // 2
        spec = {X_EDGES: (np.int32, (i.ne, 2)), X_C2N: (np.int32, (i.nc, nn)),
                X_ROWPTR: (np.int64, (i.n2 + 1,)), X_COL: (np.int32, (i.nnz_s2,)),
                X_KS: (np.float64, (i.nnz_s2,)), X_M: (np.float64, (i.nnz_s2,)),
                X_G: (np.float64, (d, i.nnz_c21)), X_MP: (np.float64, (i.nv,)),
                X_DIRNODES: (np.int32, (i.ndir,)), X_DMASK: (np.int32, (i.n2,)),
                X_LOADS: (np.float64, (i.ntraction, i.n2, d)), X_NODEXYZ: (np.float64, (i.n2, d)),
                X_C21PTR: (np.int64, (i.n2 + 1,)), X_C21COL: (np.int32, (i.nnz_c21,))}
        dt, shape = spec[which]
        out = np.zeros(max(1, int(np.prod(shape))), dt)
        _check(lib().scvs_mesh_export(self.h, which, out.ctypes.data_as(C.c_void_p)))
        return out[: int(np.prod(shape))].reshape(shape)

    def _g(self, i, ns, g):
        return _dev(g, "torch.complex128", ns * i.ndir * i.dim, self.ctx.device, "g") if g is not None else None

    def spmv(self, omega, x, y):
        i = self.info
        om, po = _host(omega, np.float64)
        n = om.size * i.ndof
        _check(lib().scvs_spmv(self.h, om.size, po, _dev(x, "torch.complex128", n, self.ctx.device, "x"),
                               _dev(y, "torch.complex128", n, self.ctx.device, "y")))

    def rhs(self, omega, traction, g, f):
        i = self.info
        om, po = _host(omega, np.float64)
        tr, pt = _traction(i, om.size, traction)
        _check(lib().scvs_rhs(self.h, om.size, po, pt, self._g(i, om.size, g),
                              _dev(f, "torch.complex128", om.size * i.ndof, self.ctx.device, "f")))

    def solve(self, omega, traction, g=None, x0=None, u=None, p=None, opts: SolveOpts | None = None):
        """Solve all systems; returns (u [nsys,n2,d], p [nsys,nv], list of Report)."""
        import torch
        i = self.info
        om, po = _host(omega, np.float64)
        ns = om.size
        tr, pt = _traction(i, ns, traction)
        dev = torch.device("cuda", self.ctx.device)
        if u is None:
            u = torch.empty((ns, i.n2, i.dim), dtype=torch.complex128, device=dev)
        if p is None:
            p = torch.empty((ns, i.nv), dtype=torch.complex128, device=dev)
        d = self.ctx.device
        pg = self._g(i, ns, g)
        px = _dev(x0, "torch.complex128", ns * i.ndof, d, "x0") if x0 is not None else None
        reps = (Report * ns)()
        o = opts if opts is not None else default_opts()
        _check(lib().scvs_solve(self.h, ns, po, pt, pg, px, _dev(u, "torch.complex128", ns * i.n2 * i.dim, d, "u"),
                                _dev(p, "torch.complex128", ns * i.nv, d, "p"), C.byref(o), reps))
        return u, p, list(reps)

    def boundary_norms(self, omega, traction, g=None):
        """Per system (traction L2(Gamma) norm^2, Dirichlet-data L2(Gamma) norm^2)."""
        i = self.info
        ns = np.asarray(omega).size
        tr, pt = _traction(i, ns, traction)
        hn2 = np.zeros(ns)
        gn2 = np.zeros(ns)
        _check(lib().scvs_boundary_norms(self.h, ns, pt, self._g(i, ns, g),
                                         hn2.ctypes.data_as(C.c_void_p), gn2.ctypes.data_as(C.c_void_p)))
        return hn2, gn2

    def mode_norms(self, u, p):
        """Per solved mode (u^H (I x M) u, p^H Mp p)."""
        i = self.info
        ns = u.shape[0]
        un2 = np.zeros(ns)
        pn2 = np.zeros(ns)
        d = self.ctx.device
        _check(lib().scvs_mode_norms(self.h, ns, _dev(u, "torch.complex128", ns * i.n2 * i.dim, d, "u"),
                                     _dev(p, "torch.complex128", ns * i.nv, d, "p"),
                                     un2.ctypes.data_as(C.c_void_p), pn2.ctypes.data_as(C.c_void_p)))
        return un2, pn2

    def mg_info(self, which: int = 0):
        """Multigrid hierarchy (0 velocity, 1 pressure): [(rows, nnz, transfer nnz)] per level."""
        n = C.c_int()
        r = np.zeros(16, np.int64)
        z = np.zeros(16, np.int64)
        q = np.zeros(16, np.int64)
        _check(lib().scvs_mesh_mg_info(self.h, which, 16, r.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p),
                                       q.ctypes.data_as(C.c_void_p), C.byref(n)))
        return [(int(r[k]), int(z[k]), int(q[k])) for k in range(min(n.value, 16))]

    def mode_norms_noalloc(self, u, p):
        """mode_norms through the entry point that allocates no device memory."""
        i = self.info
        ns = u.shape[0]
        un2 = np.zeros(ns)
        pn2 = np.zeros(ns)
        d = self.ctx.device
        _check(lib().scvs_mode_norms_noalloc(self.h, ns, _dev(u, "torch.complex128", ns * i.n2 * i.dim, d, "u"),
                                             _dev(p, "torch.complex128", ns * i.nv, d, "p"),
                                             un2.ctypes.data_as(C.c_void_p), pn2.ctypes.data_as(C.c_void_p)))
        return un2, pn2

    def autotune(self, omega, traction, g=None, base: SolveOpts | None = None):
        """Fastest of the library's candidate settings for these systems: (opts, ms)."""
        i = self.info
        om, po = _host(omega, np.float64)
        ns = om.size
        tr, pt = _traction(i, ns, traction)
        pg = self._g(i, ns, g)
        best = SolveOpts()
        ms = C.c_double()
        b = base if base is not None else default_opts()
        _check(lib().scvs_autotune(self.h, ns, po, pt, pg, C.byref(b), C.byref(best), C.byref(ms)))
        return best, ms.value


def select_modes(omega, hn2, gn2, eps, consecutive=True):
    """(order, count, e_M): the fewest modes with truncation error below eps."""
    om, po = _host(omega, np.float64)
    h, ph = _host(hn2, np.float64)
    gg, pg = _host(gn2, np.float64)
    order = np.zeros(om.size, np.int64)
    cnt = C.c_int64()
    err = C.c_double()
    _check(lib().scvs_select_modes(om.size, po, ph, pg, eps, 1 if consecutive else 0,
                                   order.ctypes.data_as(C.c_void_p), C.byref(cnt), C.byref(err)))
    return order, cnt.value, err.value


def mode_increments(omega, un2):
    """Relative L2(Omega x T) change when each mode is added to the ones before it."""
    om, po = _host(omega, np.float64)
    u, pu = _host(un2, np.float64)
    inc = np.zeros(om.size)
    _check(lib().scvs_mode_increments(om.size, po, pu, inc.ctypes.data_as(C.c_void_p)))
    return inc


def solve_groups(groups):
    """Solve several meshes' systems concurrently (each mesh on its own context and
    stream). groups: list of dicts with keys mesh, omega, traction, and optionally g,
    x0, u, p, opts. Returns [(u, p, reports)] in the same order."""
    import torch
    keep, out = [], []
    arr = (SolveGroup * len(groups))()
    for k, gr in enumerate(groups):
        m = gr["mesh"]
        i = m.info
        om, po = _host(gr["omega"], np.float64)
        ns = om.size
        tr, pt = _traction(i, ns, gr["traction"])
        dev = torch.device("cuda", m.ctx.device)
        d = m.ctx.device
        u = gr.get("u")
        p = gr.get("p")
        if u is None:
            u = torch.empty((ns, i.n2, i.dim), dtype=torch.complex128, device=dev)
        if p is None:
            p = torch.empty((ns, i.nv), dtype=torch.complex128, device=dev)
        reps = (Report * ns)()
        o = gr.get("opts") or default_opts()
        g = gr.get("g")
        x0 = gr.get("x0")
        arr[k] = SolveGroup(m.h.value if hasattr(m.h, "value") else m.h, ns, po, pt,
                            m._g(i, ns, g),
                            _dev(x0, "torch.complex128", ns * i.ndof, d, "x0") if x0 is not None else None,
                            _dev(u, "torch.complex128", ns * i.n2 * i.dim, d, "u"),
                            _dev(p, "torch.complex128", ns * i.nv, d, "p"),
                            C.cast(C.pointer(o), C.c_void_p), C.cast(reps, C.c_void_p))
        keep += [om, tr, o, reps]
        out.append((u, p, reps))
    # every group's context stream must see the inputs the caller wrote on torch's stream
    torch.cuda.synchronize()
    _check(lib().scvs_solve_groups(len(groups), C.byref(arr)))
    return [(u, p, list(r)) for u, p, r in out]


def synthesize(ctx: Context, omega, modes, times, out=None):
    """Real time samples [nt, nvals] from complex modes [nk, nvals] (device)."""
    import torch
    om, po = _host(omega, np.float64)
    tm, pt = _host(times, np.float64)
    nk = om.size
    if nk == 0 or modes.numel() % nk:
        raise ScvsError(E_INVALID, f"modes: {modes.numel()} values do not split into {nk} modes")
    nvals = modes.numel() // nk
    if out is None:
        out = torch.empty((tm.size, nvals), dtype=torch.float64, device=modes.device)
    _check(lib().scvs_synthesize(ctx.h, nk, po, _dev(modes, "torch.complex128", nk * nvals, ctx.device, "modes"),
                                 nvals, tm.size, pt, _dev(out, "torch.float64", tm.size * nvals, ctx.device, "out")))
    return out


def probe_mfma(ctx: Context, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a, pa = _host(a, np.float64)
    b, pb = _host(b, np.float64)
    d = np.zeros(256)
    _check(lib().scvs_probe_mfma(ctx.h, pa, pb, d.ctypes.data_as(C.c_void_p)))
    return d.reshape(16, 16)


class WarmStart:
    """POD + MLP warm start built from unit-amplitude mode solutions (device
    complex128 [nsnap, ndof]) at frequencies omega."""

    def __init__(self, mesh: Mesh, omega, snaps, rank=32, width=256, layers=4, seed=0):
        self.mesh = mesh
        om, po = _host(omega, np.float64)
        h = C.c_void_p()
        snp = _dev(snaps, "torch.complex128", om.size * mesh.info.ndof, mesh.ctx.device, "snaps")
        _check(lib().scvs_ws_create(mesh.h, om.size, po, snp, rank, width, layers, seed, C.byref(h)))
        self.h, self.rank, self.nsnap = h, rank, om.size

    def train(self, epochs: int, lr: float = 1e-3) -> float:
        loss = C.c_double()
        _check(lib().scvs_ws_train(self.h, epochs, lr, C.byref(loss)))
        return loss.value

    def predict(self, omega, amp, out=None):
        import torch
        om, po = _host(omega, np.float64)
        a, pa = _host(np.asarray(amp, np.complex128).view(np.float64), np.float64)
        if out is None:
            out = torch.empty((om.size, self.mesh.info.ndof), dtype=torch.complex128,
                              device=torch.device("cuda", self.mesh.ctx.device))
        if a.size != 2 * om.size:
            raise ScvsError(E_INVALID, f"amp: expected {om.size} values, got {a.size // 2}")
        _check(lib().scvs_ws_predict(self.h, om.size, po, pa, _dev(out, "torch.complex128",
                                                                    om.size * self.mesh.info.ndof,
                                                                    self.mesh.ctx.device, "out")))
        return out

    def refine(self, omega, traction, g, x0):
        """In-place minimal-residual correction of x0 over x0 + span(POD basis)."""
        om, po = _host(omega, np.float64)
        i = self.mesh.info
        tr, ptr = _traction(i, om.size, traction)
        _check(lib().scvs_ws_refine(self.h, om.size, po, ptr if i.ntraction else None, self.mesh._g(i, om.size, g),
                                    _dev(x0, "torch.complex128", om.size * i.ndof, self.mesh.ctx.device, "x0")))
        return x0

    def nparam(self) -> int:
        n = C.c_int64()
        _check(lib().scvs_ws_export(self.h, WS_NPARAM, C.byref(n)))
        return n.value

    def export(self, which: int):
        if which == WS_SIGMA:
            out = np.zeros(self.rank)
        elif which in (WS_TMEAN, WS_TSCALE):
            out = np.zeros(2 * self.rank)
        elif which == WS_PARAMS:
            out = np.zeros(self.nparam(), np.float32)
        elif which == WS_TARGETS:
            out = np.zeros((self.nsnap, 2 * self.rank), np.float32)
        elif which == WS_BASIS:
            import torch
            out = torch.empty((self.rank, self.mesh.info.ndof), dtype=torch.complex128,
                              device=torch.device("cuda", self.mesh.ctx.device))
            _check(lib().scvs_ws_export(self.h, which, _dev(out, "torch.complex128", out.numel())))
            return out
        else:
            raise ValueError(which)
        _check(lib().scvs_ws_export(self.h, which, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, params):
        p, pp = _host(params, np.float32)
        _check(lib().scvs_ws_set_params(self.h, pp))

    def loss_grad(self, x, t):
        x, px = _host(x, np.float32)
        t, pt = _host(t, np.float32)
        g = np.zeros(self.nparam(), np.float32)
        loss = C.c_double()
        _check(lib().scvs_ws_loss_grad(self.h, x.shape[0], px, pt, C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return loss.value, g

    def close(self):
        if getattr(self, "h", None):
            _check(lib().scvs_ws_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ModeWarmStarts:
    """One WarmStart per harmonic index (a POD basis per mode). Model k is built
    from unit-amplitude solutions of harmonic k at several periods, so its network
    only has to cover that harmonic's band of frequencies. `models` maps k to
    (omega [S], snaps device c128 [S, ndof]); systems are routed to the model of
    their harmonic. A group of systems whose rows are contiguous is passed as a
    view; otherwise its rows are gathered and scattered back."""

    def __init__(self, mesh: Mesh, models: dict | None = None, rank: int = 16, width: int = 256, layers: int = 4,
                 seed: int = 0):
        self.mesh, self.rank, self.width, self.layers, self.seed = mesh, rank, width, layers, seed
        self.ws = {}
        for k, (om, snaps) in (models or {}).items():
            self.add(k, om, snaps)

    def add(self, k: int, omega, snaps):
        """Model of harmonic k from its snapshots (the library copies the basis)."""
        if int(k) in self.ws:
            raise ScvsError(E_INVALID, f"harmonic {int(k)} already has a model")
        self.ws[int(k)] = WarmStart(self.mesh, omega, snaps, rank=min(self.rank, len(omega)), width=self.width,
                                    layers=self.layers, seed=self.seed + int(k))

    def train(self, schedule) -> dict:
        """schedule: [(epochs, lr), ...]; returns {k: (initial loss, final loss)}."""
        out = {}
        for k, w in self.ws.items():
            l0 = loss = w.train(0)
            for ep, lr in schedule:
                loss = w.train(ep, lr)
            out[k] = (l0, loss)
        return out

    def _groups(self, modes):
        modes = np.asarray(modes, np.int64)
        for k in np.unique(modes):
            if int(k) not in self.ws:
                raise ScvsError(E_INVALID, f"no model for harmonic {int(k)}")
            rows = np.nonzero(modes == k)[0]
            contiguous = rows[-1] - rows[0] + 1 == rows.size
            yield self.ws[int(k)], rows, (slice(int(rows[0]), int(rows[-1]) + 1) if contiguous else None)

    def predict(self, modes, omega, amp, out=None):
        import torch
        om = np.asarray(omega, np.float64)
        a = np.asarray(amp, np.complex128)
        if out is None:
            out = torch.empty((om.size, self.mesh.info.ndof), dtype=torch.complex128,
                              device=torch.device("cuda", self.mesh.ctx.device))
        for w, rows, sl in self._groups(modes):
            if sl is not None:
                w.predict(om[rows], a[rows], out=out[sl])
            else:
                out[torch.from_numpy(rows).to(out.device)] = w.predict(om[rows], a[rows])
        return out

    def refine(self, modes, omega, traction, g, x0):
        import torch
        om = np.asarray(omega, np.float64)
        tr = np.asarray(traction, np.complex128).reshape(om.size, -1)
        for w, rows, sl in self._groups(modes):
            gk = None if g is None else (g[sl] if sl is not None else g[torch.from_numpy(rows).to(g.device)].contiguous())
            if sl is not None:
                w.refine(om[rows], tr[rows], gk, x0[sl])
            else:
                idx = torch.from_numpy(rows).to(x0.device)
                x0[idx] = w.refine(om[rows], tr[rows], gk, x0[idx].contiguous())
        return x0

    def sigma(self) -> dict:
        return {k: w.export(WS_SIGMA) for k, w in self.ws.items()}

    def close(self):
        for w in self.ws.values():
            w.close()
        self.ws = {}


def herm_eig(a: np.ndarray):
    """Host Hermitian eigen-decomposition of the library (descending)."""
    a = np.ascontiguousarray(a, np.complex128)
    n = a.shape[0]
    w = np.zeros(n)
    v = np.zeros((n, n), np.complex128)
    _check(lib().scvs_herm_eig(n, a.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                               v.ctypes.data_as(C.c_void_p)))
    return w, v


def probe_mfma_bf16(ctx: Context, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a, pa = _host(a, np.float32)
    b, pb = _host(b, np.float32)
    d = np.zeros(256, np.float32)
    _check(lib().scvs_probe_mfma_bf16(ctx.h, pa, pb, d.ctypes.data_as(C.c_void_p)))
    return d.reshape(16, 16)


def version() -> str:
    return lib().scvs_version().decode()
