"""Thin Python binding of libmhdg.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; PyTorch only
provides device memory (the workspaces and vectors) and the stream.  The
method names follow the C ABI in include/mhdg.h.  If the library is missing
the binding raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhdg.so")

MHDG_FP64, MHDG_FP32, MHDG_BF16, MHDG_QELIM = 0, 1, 2, 3
MHDG_PRECONDITION, MHDG_TRANSPOSE, MHDG_GRAPH, MHDG_FOLDED = 1, 2, 4, 8
MHDG_ASSEMBLED, MHDG_BOUNDARY = 16, 32
MHDG_DRIVER_DEVICE, MHDG_DRIVER_HOST = 0, 1
MHDG_NORM_PRECONDITIONED, MHDG_NORM_TRUE = 0, 1

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "MESH", 3: "SINGULAR", 4: "NOT_CONVERGED",
          5: "WORKSPACE", 6: "HIP", 7: "STATE", 8: "NONFINITE"}

ABI_SYMBOLS = [
    "mhdg_setup_macro_mesh", "mhdg_query", "mhdg_sample_points", "mhdg_factor_local",
    "mhdg_local_matrix", "mhdg_apply_trace_operator", "mhdg_local_solve", "mhdg_rhs",
    "mhdg_solve", "mhdg_recover_local", "mhdg_destroy", "mhdg_last_error",
    "mhdg_status_string", "mhdg_profile", "mhdg_mass_apply", "mhdg_adjoint",
    "mhdg_set_instances", "mhdg_factor_local_batched", "mhdg_autotune",
    "mhdg_set_kernel_variant", "mhdg_fold_operator", "mhdg_apply_many_ws_bytes",
    "mhdg_apply_trace_operator_many", "mhdg_flux_balance", "mhdg_set_supg",
    "mhdg_apply_trace_operator_many_noalloc", "mhdg_trace_matrix_ws_bytes",
    "mhdg_assemble_trace_matrix", "mhdg_boundary_ws_bytes", "mhdg_condense_boundary",
]
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024
MHDG_TUNE_LU, MHDG_TUNE_SOLVE = 1, 2
MAX_CLASSES = 8


class MhdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Sizes(ctypes.Structure):
    _fields_ = [("n_macro", ctypes.c_int64), ("n_faces", ctypes.c_int64),
                ("n_interior_faces", ctypes.c_int64), ("n_trace", ctypes.c_int64),
                ("n_nodes", ctypes.c_int64), ("n_local", ctypes.c_int64),
                ("n_bnd_points", ctypes.c_int64), ("p", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("max_local", ctypes.c_int64),
                ("factor_ws_bytes", ctypes.c_size_t), ("solve_ws_bytes", ctypes.c_size_t),
                ("n_instances", ctypes.c_int32), ("fold_ws_bytes", ctypes.c_size_t)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("zero_guess", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("graph", ctypes.c_int32), ("folded", ctypes.c_int32),
                ("classic_gs", ctypes.c_int32), ("driver", ctypes.c_int32),
                ("stop_norm", ctypes.c_int32), ("assembled", ctypes.c_int32),
                ("boundary", ctypes.c_int32)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32 * 6), ("ms", ctypes.c_double * 6)]
    NAMES = ("assemble", "lu", "apply_macro_solve", "face_combine", "other_macro_solve",
             "folded_apply")

    def as_dict(self):
        return {n: {"count": int(self.count[i]), "ms": float(self.ms[i])}
                for i, n in enumerate(self.NAMES)}


class TuneReport(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int32), ("N", ctypes.c_int32 * 8),
                ("count", ctypes.c_int64 * 8), ("lu_variant", ctypes.c_int32 * 8),
                ("solve_variant", ctypes.c_int32 * 8), ("lu_ms", (ctypes.c_double * 6) * 8),
                ("apply_ms", (ctypes.c_double * 8) * 8)]

    def as_list(self):
        out = []
        for i in range(self.n_classes):
            out.append({"N": int(self.N[i]), "count": int(self.count[i]),
                        "lu_variant": int(self.lu_variant[i]),
                        "solve_variant": int(self.solve_variant[i]),
                        "lu_ms": {v: float(self.lu_ms[i][v]) for v in range(1, 6) if self.lu_ms[i][v]},
                        "apply_ms": {v: float(self.apply_ms[i][v]) for v in range(1, 8)
                                     if self.apply_ms[i][v]}})
        return out


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_res_prec", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("t_rhs_ms", ctypes.c_double), ("t_gmres_ms", ctypes.c_double),
                ("n_applies", ctypes.c_int32), ("outer_iterations", ctypes.c_int32),
                ("reorth_passes", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("host_waits", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmhdg.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "(the HIP library is required, there is no fallback)")
    lib = ctypes.CDLL(path)
    P, I32, I64, D, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                          ctypes.c_size_t)
    sig = {
        "mhdg_setup_macro_mesh": [I64, P, I64, P, P, I32, I32, ctypes.POINTER(P)],
        "mhdg_query": [P, I32, I32, ctypes.POINTER(Sizes)],
        "mhdg_sample_points": [P, P, P],
        "mhdg_factor_local": [P, P, D, D, D, I32, P, SZ, P],
        "mhdg_factor_local_batched": [P, P, P, D, I32, P, SZ, P],
        "mhdg_set_instances": [P, I32],
        "mhdg_autotune": [P, I32, ctypes.POINTER(TuneReport), P],
        "mhdg_set_kernel_variant": [P, I32, I32, I32],
        "mhdg_set_supg": [P, I32],
        "mhdg_fold_operator": [P, P, SZ, P],
        "mhdg_assemble_trace_matrix": [P, P, SZ, P],
        "mhdg_condense_boundary": [P, P, SZ, P],
        "mhdg_local_matrix": [P, I64, P, P],
        "mhdg_apply_trace_operator": [P, P, P, I32, P],
        "mhdg_apply_trace_operator_many": [P, I32, P, P, I32, P, SZ, P],
        "mhdg_apply_trace_operator_many_noalloc": [P, I32, P, P, I32, P],
        "mhdg_local_solve": [P, P, P, I32, P],
        "mhdg_rhs": [P, P, P, P, I32, P],
        "mhdg_solve": [P, P, P, ctypes.POINTER(SolveOpts), P, P, SZ, P, P],
        "mhdg_recover_local": [P, P, P, P, P],
        "mhdg_flux_balance": [P, P, P, P, P, P],
        "mhdg_profile": [P, I32, ctypes.POINTER(KernelTimes)],
        "mhdg_mass_apply": [P, P, P, P],
        "mhdg_adjoint": [P, P, P, P, ctypes.POINTER(SolveOpts), P, P, P, P, P, SZ,
                         ctypes.POINTER(SolveInfo), P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mhdg_apply_many_ws_bytes.argtypes = [P, I32]
    lib.mhdg_apply_many_ws_bytes.restype = SZ
    lib.mhdg_trace_matrix_ws_bytes.argtypes = [P]
    lib.mhdg_trace_matrix_ws_bytes.restype = SZ
    lib.mhdg_boundary_ws_bytes.argtypes = [P]
    lib.mhdg_boundary_ws_bytes.restype = SZ
    lib.mhdg_destroy.argtypes = [P]
    lib.mhdg_destroy.restype = None
    lib.mhdg_last_error.argtypes = [P]
    lib.mhdg_last_error.restype = ctypes.c_char_p
    lib.mhdg_status_string.argtypes = [I32]
    lib.mhdg_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


class MacroMesh:
    """Handle of a macro mesh on the library side, plus the torch workspaces
    that hold its factors (kept alive for as long as the handle uses them)."""

    def __init__(self, xy, tri, level, p: int):
        lib = load_library()
        self._lib = lib
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        if np.ndim(level) == 0:
            lev_arr, uniform = None, int(level)
        else:
            lev_arr, uniform = np.ascontiguousarray(level, dtype=np.int32), 0
        h = ctypes.c_void_p()
        st = lib.mhdg_setup_macro_mesh(xy.shape[0], xy.ctypes.data, tri.shape[0], tri.ctypes.data,
                                       None if lev_arr is None else lev_arr.ctypes.data, uniform,
                                       int(p), ctypes.byref(h))
        if st != 0:
            raise MhdgError(st, "setup_macro_mesh rejected the mesh")
        self.h = h
        self._level = (np.full(tri.shape[0], uniform, dtype=np.int64) if lev_arr is None
                       else lev_arr.astype(np.int64))
        self._p = int(p)
        self.factor_ws = None
        self.solve_ws = None
        self.precision = MHDG_FP64
        self.sizes = self.query()
        # bumped by every call that changes the factors, the folded operators or
        # the stored local right-hand sides (lets wrappers tell whether the
        # handle still holds the state they left in it)
        self.state_gen = 0

    def close(self):
        """Destroy the library handle (its device tables, graphs and private
        stream) and drop the workspaces; the object is unusable afterwards."""
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._lib.mhdg_destroy(h)
        self.h = None
        self.factor_ws = self.solve_ws = self.fold_ws = self.many_ws = None
        self.matrix_ws = self.boundary_ws = None

    def __del__(self):
        self.close()

    def _check(self, st, what):
        if st != 0:
            msg = self._lib.mhdg_last_error(self.h).decode()
            raise MhdgError(st, f"{what}: {msg}")

    # ---- C ABI calls ---------------------------------------------------
    def query(self, precision=MHDG_FP64, restart=30) -> Sizes:
        s = Sizes()
        self._check(self._lib.mhdg_query(self.h, precision, restart, ctypes.byref(s)), "query")
        return s

    def set_instances(self, n_inst: int):
        """n_inst coefficient instances in one handle (instance-major vectors)."""
        self.state_gen += 1
        self._check(self._lib.mhdg_set_instances(self.h, int(n_inst)), "set_instances")
        self.sizes = self.query()
        self.factor_ws = None
        self.solve_ws = None

    @property
    def n_instances(self) -> int:
        return int(self.sizes.n_instances)

    def macro_P(self):
        """P = 2^r_K p of every macro (all instances, instance-major)."""
        return np.tile((2 ** self._level) * self._p, self.n_instances)

    def sample_points(self):
        s = self.sizes
        node = np.zeros((s.n_nodes, 2))
        bnd = np.zeros((max(s.n_bnd_points, 1), 2))
        self._check(self._lib.mhdg_sample_points(self.h, node.ctypes.data, bnd.ctypes.data),
                    "sample_points")
        return node, bnd[:s.n_bnd_points]

    def factor_local(self, kappa, beta, tau=1.0, precision=MHDG_FP64, stream=None):
        self.state_gen += 1
        import torch
        s = self.query(precision)
        if self.factor_ws is None or self.factor_ws.numel() < s.factor_ws_bytes:
            self.factor_ws = None
            self.factor_ws = torch.empty(s.factor_ws_bytes, dtype=torch.uint8, device="cuda")
        kap = torch.as_tensor(kappa, dtype=torch.float64, device="cuda")
        if kap.ndim == 0:
            kap = kap.expand(s.n_macro)
        kap = kap.reshape(-1).contiguous()
        if kap.numel() != s.n_macro:
            raise ValueError(f"kappa has {kap.numel()} values, expected {s.n_macro}")
        self._kappa = kap
        self.precision = precision
        b = np.ascontiguousarray(beta, dtype=np.float64)
        if b.size == 2:
            self._check(self._lib.mhdg_factor_local(self.h, _ptr(kap), float(b.flat[0]),
                                                    float(b.flat[1]), float(tau), precision,
                                                    _ptr(self.factor_ws), self.factor_ws.numel(),
                                                    _stream(stream)), "factor_local")
            return
        if b.size != 2 * s.n_instances:
            raise ValueError(f"beta must hold 2 or 2 x {s.n_instances} values")
        self._check(self._lib.mhdg_factor_local_batched(self.h, _ptr(kap), b.ctypes.data,
                                                        float(tau), precision,
                                                        _ptr(self.factor_ws),
                                                        self.factor_ws.numel(), _stream(stream)),
                    "factor_local_batched")

    def local_matrix(self, e, out, stream=None):
        self._check(self._lib.mhdg_local_matrix(self.h, int(e), _ptr(out), _stream(stream)),
                    "local_matrix")

    def apply_trace_operator(self, lam, out, flags=0, stream=None):
        self._check(self._lib.mhdg_apply_trace_operator(self.h, _ptr(lam), _ptr(out), flags,
                                                        _stream(stream)), "apply_trace_operator")

    def apply_trace_operator_many(self, lam, out, flags=0, stream=None):
        """out[v] = S lam[v] (D^-1 S lam[v] with MHDG_PRECONDITION) for every row v
        of the contiguous device tensors lam, out of shape (n_rhs, n_trace)."""
        import torch
        n_rhs = int(lam.shape[0]) if lam.dim() == 2 else 1
        need = int(self._lib.mhdg_apply_many_ws_bytes(self.h, n_rhs))
        if getattr(self, "many_ws", None) is None or self.many_ws.numel() < need:
            self.many_ws = None
            self.many_ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        self._check(self._lib.mhdg_apply_trace_operator_many(
            self.h, n_rhs, _ptr(lam), _ptr(out), flags, _ptr(self.many_ws), self.many_ws.numel(),
            _stream(stream)), "apply_trace_operator_many")

    def apply_many_ws_bytes(self, n_rhs):
        """Bytes of contribution slots a many-vector apply of n_rhs vectors needs."""
        return int(self._lib.mhdg_apply_many_ws_bytes(self.h, int(n_rhs)))

    def apply_trace_operator_many_noalloc(self, lam, out, flags=0, stream=None):
        """The same as apply_trace_operator_many with the library's fixed
        per-GPU scratch instead of a workspace (no device allocation; calls
        on one GPU must not overlap)."""
        n_rhs = int(lam.shape[0]) if lam.dim() == 2 else 1
        self._check(self._lib.mhdg_apply_trace_operator_many_noalloc(
            self.h, n_rhs, _ptr(lam), _ptr(out), flags, _stream(stream)),
            "apply_trace_operator_many_noalloc")

    def local_solve(self, x, y, flags=0, stream=None):
        self._check(self._lib.mhdg_local_solve(self.h, _ptr(x), _ptr(y), flags, _stream(stream)),
                    "local_solve")

    def rhs(self, f_nodes, g_bnd, fhat, flags=0, stream=None):
        self.state_gen += 1
        self._check(self._lib.mhdg_rhs(self.h, _ptr(f_nodes), _ptr(g_bnd), _ptr(fhat), flags,
                                       _stream(stream)), "rhs")

    def solve(self, f_nodes, g_bnd, lam, rtol=1e-10, restart=30, max_iter=10000, zero_guess=True,
              stream=None, check=True, inner_rtol=0.0, max_outer=0, graph=True, folded=False,
              classic_gs=False, driver=None, stop_norm=None, assembled=False, boundary=False):
        import torch
        self.state_gen += 1
        s = self.query(self.precision, restart)
        if self.solve_ws is None or self.solve_ws.numel() < s.solve_ws_bytes:
            self.solve_ws = None
            self.solve_ws = torch.empty(s.solve_ws_bytes, dtype=torch.uint8, device="cuda")
        opts = SolveOpts(float(rtol), int(restart), int(max_iter), 1 if zero_guess else 0,
                         int(max_outer), float(inner_rtol), 1 if graph else 0,
                         1 if folded else 0, 1 if classic_gs else 0,
                         MHDG_DRIVER_DEVICE if driver is None else int(driver),
                         MHDG_NORM_PRECONDITIONED if stop_norm is None else int(stop_norm),
                         1 if assembled else 0, 1 if boundary else 0)
        infos = (SolveInfo * max(1, s.n_instances))()
        st = self._lib.mhdg_solve(self.h, _ptr(f_nodes), _ptr(g_bnd), ctypes.byref(opts), _ptr(lam),
                                  _ptr(self.solve_ws), self.solve_ws.numel(),
                                  ctypes.cast(infos, ctypes.c_void_p), _stream(stream))
        self.last_solve_info = infos[0].as_dict()
        self.last_solve_infos = [i.as_dict() for i in infos]
        if check:
            self._check(st, "solve")
        return infos[0]

    def mass_apply(self, v, out, stream=None):
        self._check(self._lib.mhdg_mass_apply(self.h, _ptr(v), _ptr(out), _stream(stream)),
                    "mass_apply")

    def adjoint(self, lam, qu, dJ_dU, psi_lam, psi_U, dJ_dkappa, dJ_dbeta, rtol=1e-12,
                restart=300, max_iter=20000, stream=None, graph=True, folded=False,
                classic_gs=False, driver=None, boundary=False):
        import torch
        s = self.query(self.precision, restart)
        if self.solve_ws is None or self.solve_ws.numel() < s.solve_ws_bytes:
            self.solve_ws = None
            self.solve_ws = torch.empty(s.solve_ws_bytes, dtype=torch.uint8, device="cuda")
        opts = SolveOpts(float(rtol), int(restart), int(max_iter), 1, 0, 0.0, 1 if graph else 0,
                         1 if folded else 0, 1 if classic_gs else 0,
                         MHDG_DRIVER_DEVICE if driver is None else int(driver),
                         MHDG_NORM_PRECONDITIONED, 0, 1 if boundary else 0)
        info = SolveInfo()
        self._check(self._lib.mhdg_adjoint(self.h, _ptr(lam), _ptr(qu), _ptr(dJ_dU),
                                           ctypes.byref(opts), _ptr(psi_lam), _ptr(psi_U),
                                           _ptr(dJ_dkappa), _ptr(dJ_dbeta), _ptr(self.solve_ws),
                                           self.solve_ws.numel(), ctypes.byref(info),
                                           _stream(stream)), "adjoint")
        self.last_adjoint_info = info.as_dict()
        return info

    def autotune(self, flags=MHDG_TUNE_LU | MHDG_TUNE_SOLVE, stream=None):
        """Time the kernel variants per size class on this handle's data and
        keep the fastest; returns the per-class report."""
        self.state_gen += 1
        rep = TuneReport()
        self._check(self._lib.mhdg_autotune(self.h, int(flags), ctypes.byref(rep),
                                            _stream(stream)), "autotune")
        return rep.as_list()

    def fold_operator(self, stream=None):
        """Build the folded macro operators T_K = C_K A_K^-1 B_K (FP64 factors
        needed); then apply/solve can use them (MHDG_FOLDED / folded=True)."""
        self.state_gen += 1
        import torch
        s = self.query(self.precision)
        if getattr(self, "fold_ws", None) is None or self.fold_ws.numel() < s.fold_ws_bytes:
            self.fold_ws = None
            self.fold_ws = torch.empty(max(s.fold_ws_bytes, 1), dtype=torch.uint8, device="cuda")
        self._check(self._lib.mhdg_fold_operator(self.h, _ptr(self.fold_ws), self.fold_ws.numel(),
                                                 _stream(stream)), "fold_operator")

    def assemble_trace_matrix(self, stream=None):
        """Assemble the global trace matrix S from the folded operators (call
        fold_operator first); then apply/solve can use it (MHDG_ASSEMBLED /
        assembled=True)."""
        self.state_gen += 1
        import torch
        need = int(self._lib.mhdg_trace_matrix_ws_bytes(self.h))
        if getattr(self, "matrix_ws", None) is None or self.matrix_ws.numel() < need:
            self.matrix_ws = None
            self.matrix_ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        self._check(self._lib.mhdg_assemble_trace_matrix(self.h, _ptr(self.matrix_ws),
                                                         self.matrix_ws.numel(), _stream(stream)),
                    "assemble_trace_matrix")

    def condense_boundary(self, stream=None):
        """Boundary-condensed blocks W_K = (A_K^-1)_bb of every macro from the
        FP64 factors (call factor_local first); then apply/solve/adjoint can
        use them (MHDG_BOUNDARY / boundary=True)."""
        self.state_gen += 1
        import torch
        need = int(self._lib.mhdg_boundary_ws_bytes(self.h))
        if getattr(self, "boundary_ws", None) is None or self.boundary_ws.numel() < need:
            self.boundary_ws = None
            self.boundary_ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        self._check(self._lib.mhdg_condense_boundary(self.h, _ptr(self.boundary_ws),
                                                     self.boundary_ws.numel(), _stream(stream)),
                    "condense_boundary")

    def boundary_blocks(self):
        """The blocks of condense_boundary as a list of FP64 (9P x 9P) device
        views, W_K[row, col] (the workspace layout of mhdg_condense_boundary)."""
        import torch
        n = int(self.sizes.n_macro)
        ws = self.boundary_ws
        off = ws[:8 * n].view(torch.int64).cpu()
        base = (8 * n + 255) // 256 * 256
        W = ws[base:].view(torch.float64)
        out = []
        for e, P in enumerate(self.macro_P()):
            nb = 9 * int(P)
            o = int(off[e])
            out.append(W[o:o + nb * nb].view(nb, nb).t())
        return out

    def set_supg(self, on: bool):
        """SUPG stabilisation inside the macros (section 3.4) on or off; the
        factors must be computed again afterwards."""
        self.state_gen += 1
        self._check(self._lib.mhdg_set_supg(self.h, 1 if on else 0), "set_supg")

    def set_kernel_variant(self, N, lu_variant=0, solve_variant=0):
        self._check(self._lib.mhdg_set_kernel_variant(self.h, int(N), int(lu_variant),
                                                      int(solve_variant)), "set_kernel_variant")

    def profile(self, enable: bool):
        """Start (True) or stop (False) per-kernel event timing; stop returns
        the accumulated counts and milliseconds per kernel class."""
        kt = KernelTimes()
        self._check(self._lib.mhdg_profile(self.h, 1 if enable else 0, ctypes.byref(kt)), "profile")
        return None if enable else kt.as_dict()

    def flux_balance(self, lam, qu, f_nodes, out, stream=None):
        """out[K] = <flux^.n, 1>_dK - (f_h, 1)_K for every macro (device f64[n_macro])."""
        self._check(self._lib.mhdg_flux_balance(self.h, _ptr(lam), _ptr(qu), _ptr(f_nodes),
                                                _ptr(out), _stream(stream)), "flux_balance")

    def recover_local(self, lam, qu, flux_res=None, stream=None):
        self._check(self._lib.mhdg_recover_local(self.h, _ptr(lam), _ptr(qu), _ptr(flux_res),
                                                 _stream(stream)), "recover_local")


def setup_macro_mesh(xy, tri, level, p) -> MacroMesh:
    return MacroMesh(xy, tri, level, p)
