"""ctypes binding of libpcloth.so: argument marshalling only.

Every computation runs in the HIP library.  If the library is missing the
import fails; there is no fallback path.  Device buffers are torch tensors on
``cuda:0`` (float64, shape (nv, 3), contiguous); the current torch stream is
passed to every call.  By default the library's own device memory comes from
torch's caching allocator (pc_set_allocator), so the library and torch share
one pool.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcloth.so")

PC_OK, PC_ERR_ARG, PC_ERR_MESH, PC_ERR_HIP, PC_ERR_OOM, PC_ERR_NONFINITE, PC_ERR_NOT_CONVERGED, \
    PC_ERR_CAPACITY = range(8)
STATUS_NAMES = {0: "PC_OK", 1: "PC_ERR_ARG", 2: "PC_ERR_MESH", 3: "PC_ERR_HIP", 4: "PC_ERR_OOM",
                5: "PC_ERR_NONFINITE", 6: "PC_ERR_NOT_CONVERGED", 7: "PC_ERR_CAPACITY"}
PC_F64, PC_F32, PC_BF16, PC_F16 = 0, 1, 2, 3
DTYPES = {"f64": PC_F64, "f32": PC_F32, "bf16": PC_BF16, "f16": PC_F16}

# Names of every entry point declared in include/pcloth.h.
ABI_SYMBOLS = ["pc_create", "pc_destroy", "pc_set_params", "pc_last_error", "pc_sizes", "pc_get_hinges",
               "cloth_assemble", "cloth_pcg_solve", "cloth_step", "cloth_spmv", "cloth_export_blocks",
               "cloth_export_pattern", "pc_check", "pc_profile", "pc_profile_read", "pc_set_option",
               "pc_ws_set_params", "pc_ws_get_params", "pc_ws_features", "pc_ws_predict", "pc_ws_gradient",
               "pc_ws_train_step", "pc_mfma_probe", "pc_get_option", "pc_set_instances", "pc_get_instance_info",
               "pc_autotune", "cloth_export_precond", "pc_ws_start", "cloth_set_contacts",
               "cloth_assemble_bell", "cloth_spmv_bell", "cloth_export_bell", "pc_set_allocator",
               "pc_ws_predict_noalloc"]
WS_PARAMS = 10307
# Warm-start network layer shapes (inputs x outputs); the flat parameter
# vector holds, per layer, W row-major then the bias.
WS_SHAPES = [(27, 64), (64, 64), (64, 64), (64, 3)]
WARM = {"zero": 0, "prev": 1, "given": 1, "learned": 2}
METHOD = {"cg": 0, "chronopoulos-gear": 1}
PC_OPT_GRAPH_CHUNK, PC_OPT_SPMV_SLICES_PER_BLOCK, PC_OPT_VECTOR_ROWS_PER_BLOCK, PC_OPT_LDS_WINDOW, \
    PC_OPT_NARROW_COLUMNS, PC_OPT_SPMV_NARROW_ACTIVE, PC_OPT_INNER_FP32, PC_OPT_KEEP_DIRECTION = 0, 1, 2, 3, 4, 5, 6, 7
PROFILE_KINDS = ["spmv", "cg_update", "cg_dir", "row_assemble", "row_pattern", "assemble_all", "elements", "k7"]


class PcParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("mu", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("k_bend", ctypes.c_double), ("beta", ctypes.c_double), ("gravity", ctypes.c_double * 3),
                ("rhs_mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PcMesh(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("nt", ctypes.c_int32), ("tris", ctypes.POINTER(ctypes.c_int32)),
                ("rest", ctypes.POINTER(ctypes.c_double)), ("mass", ctypes.POINTER(ctypes.c_double)),
                ("pinned", ctypes.POINTER(ctypes.c_uint8))]


class PcBsr3(ctypes.Structure):
    _fields_ = [("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("dtype", ctypes.c_int),
                ("nrows", ctypes.c_int32), ("nnzb", ctypes.c_int32)]


class PcSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_rho", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("warm", ctypes.c_int32), ("check_every", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("method", ctypes.c_int32)]


PRECOND = {"jacobi": 0, "block": 1}


def solve_opts(tol=1e-6, maxit=20000, warm=False, check_every=0, inner_rho=0.0, max_sweeps=0, precond="jacobi",
               method="cg"):
    w = WARM[warm] if isinstance(warm, str) else int(warm)
    pre = PRECOND[precond] if isinstance(precond, str) else int(precond)
    m = METHOD[method] if isinstance(method, str) else int(method)
    return PcSolveOpts(float(tol), float(inner_rho), int(maxit), w, int(check_every), int(max_sweeps), pre, m)


class PcSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("rel_res_recursive", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("bnorm", ctypes.c_double), ("fallback", ctypes.c_int32),
                ("warm_used", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "sweeps": self.sweeps, "rel_res_recursive": self.rel_res_recursive,
                "rel_res_true": self.rel_res_true, "bnorm": self.bnorm, "fallback": self.fallback,
                "warm_used": self.warm_used}


_lib = None


def lib():
    """Load libpcloth.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2008_00409_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.pc_create.argtypes = [ctypes.POINTER(PcMesh), ctypes.POINTER(PcParams), ctypes.POINTER(vp)]
        L.pc_destroy.argtypes = [vp]
        L.pc_set_params.argtypes = [vp, ctypes.POINTER(PcParams)]
        L.pc_last_error.argtypes = [vp]
        L.pc_last_error.restype = ctypes.c_char_p
        L.pc_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.pc_get_hinges.argtypes = [vp, vp, vp]
        L.cloth_assemble.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(PcBsr3), vp, vp, vp]
        L.cloth_pcg_solve.argtypes = [vp, vp, vp, ctypes.POINTER(PcSolveOpts), ctypes.POINTER(PcSolveInfo), vp]
        L.cloth_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(PcSolveOpts),
                                 ctypes.POINTER(PcSolveInfo), vp]
        L.cloth_spmv.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
        L.cloth_export_blocks.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
        L.cloth_export_precond.argtypes = [vp, vp, vp, vp]
        L.cloth_set_contacts.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp]
        L.pc_check.argtypes = [vp, vp]
        L.cloth_assemble_bell.argtypes = [vp, vp, vp, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_int32), vp]
        L.cloth_spmv_bell.argtypes = [vp, vp, vp, vp]
        L.cloth_export_bell.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp, vp, vp]
        L.cloth_export_pattern.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp]
        L.pc_profile.argtypes = [vp, ctypes.c_int32]
        L.pc_set_option.argtypes = [vp, ctypes.c_int32, ctypes.c_int64]
        L.pc_ws_set_params.argtypes = [vp, vp, ctypes.c_int32]
        L.pc_ws_get_params.argtypes = [vp, vp, ctypes.c_int32]
        L.pc_ws_features.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.pc_ws_predict.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.pc_ws_predict_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.pc_ws_start.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
        L.pc_ws_gradient.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
        L.pc_ws_train_step.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
        L.pc_mfma_probe.argtypes = [vp, vp]
        L.pc_get_option.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        L.pc_set_instances.argtypes = [vp, vp, ctypes.c_int32]
        L.pc_get_instance_info.argtypes = [vp, ctypes.POINTER(PcSolveInfo), ctypes.c_int32]
        L.pc_autotune.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_double), vp]
        L.pc_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.pc_set_allocator.argtypes = [vp, _ALLOC_FN, _FREE_FN, vp]
        for name in ABI_SYMBOLS:
            if name not in ("pc_last_error",):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """torch's caching allocator as the library's device allocator
    (pc_set_allocator).  Counts the blocks it hands out and takes back."""

    def __init__(self):
        self.live = {}
        self.n_alloc = 0
        self.n_free = 0
        self.bytes = 0
        self.alloc_fn = _ALLOC_FN(self._alloc)
        self.free_fn = _FREE_FN(self._free)

    def _alloc(self, nbytes, _user):
        try:
            import torch
            ptr = int(torch.cuda.caching_allocator_alloc(int(nbytes)))
        except Exception:      # the library turns NULL into PC_ERR_OOM
            return None
        self.live[ptr] = int(nbytes)
        self.n_alloc += 1
        self.bytes += int(nbytes)
        return ptr

    def _free(self, ptr, _user):
        self.live.pop(ptr, None)
        self.n_free += 1
        try:
            import torch
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass


_TORCH_ALLOCATOR = None


def torch_allocator():
    """The process-wide TorchAllocator the contexts use by default."""
    global _TORCH_ALLOCATOR
    if _TORCH_ALLOCATOR is None:
        _TORCH_ALLOCATOR = TorchAllocator()
    return _TORCH_ALLOCATOR


# Contexts still open at interpreter exit are closed while torch (whose
# allocator takes their memory back) is still usable.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for c in list(_LIVE):
        try:
            c.close()
        except Exception:
            pass


class PclothError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _dev3(t, nv, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and tuple(t.shape) == (nv, 3)):
        raise ValueError(f"{name} must be a contiguous cuda float64 tensor of shape ({nv}, 3)")
    return _ptr(t)


def make_params(h, mu=1000.0, lam=500.0, k_bend=1e-5, beta=0.0, gravity=(0.0, 0.0, -9.81), rhs_mode=1):
    p = PcParams()
    p.h, p.mu, p.lambda_, p.k_bend, p.beta = float(h), float(mu), float(lam), float(k_bend), float(beta)
    for a in range(3):
        p.gravity[a] = float(gravity[a])
    p.rhs_mode = int(rhs_mode)
    return p


class Context:
    """One cloth on the GPU: wraps pc_create / pc_destroy and the step calls."""

    def __init__(self, rest, tris, mass, pinned, params: PcParams, allocator="torch"):
        """allocator: "torch" (torch's caching allocator, the default), None
        (hipMalloc inside the library) or a TorchAllocator-like object with
        alloc_fn / free_fn ctypes callbacks."""
        L = lib()
        if allocator == "torch":
            allocator = torch_allocator()
        self.allocator = allocator
        if allocator is None:
            L.pc_set_allocator(None, _ALLOC_FN(), _FREE_FN(), None)
        else:
            L.pc_set_allocator(None, allocator.alloc_fn, allocator.free_fn, None)
        self._keep = [np.ascontiguousarray(rest, dtype=np.float64),
                      np.ascontiguousarray(tris, dtype=np.int32),
                      np.ascontiguousarray(mass, dtype=np.float64),
                      np.ascontiguousarray(pinned, dtype=np.uint8)]
        rest_, tris_, mass_, pin_ = self._keep
        m = PcMesh()
        m.nv, m.nt = rest_.shape[0], tris_.shape[0]
        m.tris = tris_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        m.rest = rest_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        m.mass = mass_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        m.pinned = pin_.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self.params = params
        h = ctypes.c_void_p()
        st = L.pc_create(ctypes.byref(m), ctypes.byref(params), ctypes.byref(h))
        if st != PC_OK:
            raise PclothError(st, L.pc_last_error(None).decode())
        self.h = h
        _LIVE.add(self)
        self.nv, self.nt = int(m.nv), int(m.nt)
        sz = (ctypes.c_int64 * 4)()
        L.pc_sizes(self.h, sz)
        self.nh, self.cap = int(sz[2]), int(sz[3])

    @classmethod
    def from_cloth(cls, c, allocator="torch", **kw):
        return cls(c.rest, c.tris, c.mass, c.pinned, make_params(c.h, **kw), allocator=allocator)

    def close(self):
        if getattr(self, "h", None):
            lib().pc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != PC_OK:
            raise PclothError(st, lib().pc_last_error(self.h).decode())

    # -- entry points -------------------------------------------------------
    def set_params(self, params: PcParams):
        self._check(lib().pc_set_params(self.h, ctypes.byref(params)))
        self.params = params

    def hinges(self):
        H = np.zeros((self.nh, 4), dtype=np.int32)
        C = np.zeros((self.nh, 2), dtype=np.float64)
        self._check(lib().pc_get_hinges(self.h, H.ctypes.data_as(ctypes.c_void_p),
                                        C.ctypes.data_as(ctypes.c_void_p)))
        return H, C

    def cloth_assemble(self, x, v, dtype="f32", b=None, diag=None):
        import torch
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        if b is None:
            b = torch.empty((self.nv, 3), dtype=torch.float64, device=x.device)
        A = PcBsr3()
        self._check(lib().cloth_assemble(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"), dt,
                                         ctypes.byref(A), _dev3(b, self.nv, "b"),
                                         _dev3(diag, self.nv, "diag") if diag is not None else None, _stream()))
        self._A = A
        return b

    def pattern(self):
        """Block-CSR pattern of the last assembly as torch int32 tensors (rowptr, colidx)."""
        import torch
        n = ctypes.c_int64()
        self._check(lib().cloth_export_pattern(self.h, None, None, ctypes.byref(n), _stream()))
        rowptr = torch.empty(self.nv + 1, dtype=torch.int32, device="cuda")
        colidx = torch.empty(max(1, n.value), dtype=torch.int32, device="cuda")
        self._check(lib().cloth_export_pattern(self.h, _ptr(rowptr), _ptr(colidx), None, _stream()))
        return rowptr, colidx[:n.value]

    def cloth_pcg_solve(self, b, dv=None, tol=1e-6, maxit=20000, warm=False, check_every=0, raise_on_error=True,
                        inner_rho=0.0, max_sweeps=0, precond="jacobi", method="cg"):
        import torch
        if dv is None:
            dv = torch.zeros((self.nv, 3), dtype=torch.float64, device=b.device)
        o = solve_opts(tol, maxit, warm, check_every, inner_rho, max_sweeps, precond, method)
        info = PcSolveInfo()
        st = lib().cloth_pcg_solve(self.h, _dev3(b, self.nv, "b"), _dev3(dv, self.nv, "dv"), ctypes.byref(o),
                                   ctypes.byref(info), _stream())
        if raise_on_error:
            self._check(st)
        d = info.as_dict()
        d["status"] = st
        return dv, d

    def cloth_spmv(self, x, y=None, solver_blocks=False):
        import torch
        if y is None:
            y = torch.empty_like(x)
        self._check(lib().cloth_spmv(self.h, _dev3(x, self.nv, "x"), _dev3(y, self.nv, "y"), int(solver_blocks),
                                     _stream()))
        return y

    def cloth_set_contacts(self, verts=None, weights=None, normals=None, thickness=0.0, stiffness=0.0):
        """Proximity pairs for the following assemblies (None: remove them).
        Arrays may be numpy or torch; they are copied to the device first."""
        import torch
        if verts is None or len(verts) == 0:
            self._check(lib().cloth_set_contacts(self.h, 0, None, None, None, 0.0, 0.0, _stream()))
            return
        v = torch.as_tensor(np.ascontiguousarray(verts, dtype=np.int32) if isinstance(verts, np.ndarray) else verts,
                            dtype=torch.int32, device="cuda").contiguous()
        w = torch.as_tensor(weights, dtype=torch.float64, device="cuda").contiguous()
        n = torch.as_tensor(normals, dtype=torch.float64, device="cuda").contiguous()
        nc = v.shape[0]
        if v.shape != (nc, 4) or w.shape != (nc, 4) or n.shape != (nc, 3):
            raise ValueError("contacts: verts (nc, 4), weights (nc, 4), normals (nc, 3)")
        self._check(lib().cloth_set_contacts(self.h, int(nc), _ptr(v), _ptr(w), _ptr(n), float(thickness),
                                             float(stiffness), _stream()))

    def cloth_export_precond(self):
        """(1 / diag(A) as (nv, 3), inverse diagonal blocks as (nv, 3, 3)), float32 on the device."""
        import torch
        dinv = torch.empty((self.nv, 3), dtype=torch.float32, device="cuda")
        b6 = torch.empty((self.nv, 6), dtype=torch.float32, device="cuda")
        self._check(lib().cloth_export_precond(self.h, _ptr(dinv), _ptr(b6), _stream()))
        idx = [0, 1, 2, 1, 3, 4, 2, 4, 5]
        return dinv, b6[:, idx].reshape(self.nv, 3, 3)

    def cloth_assemble_bell(self, x, v, dtype="f32", b=None):
        """The paper's five-step filling into a BELL table: returns (b, width)."""
        import torch
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        if b is None:
            b = torch.empty((self.nv, 3), dtype=torch.float64, device="cuda")
        w = ctypes.c_int32(0)
        self._check(lib().cloth_assemble_bell(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"), dt,
                                              _dev3(b, self.nv, "b"), ctypes.byref(w), _stream()))
        return b, int(w.value)

    def cloth_spmv_bell(self, x, y=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        self._check(lib().cloth_spmv_bell(self.h, _dev3(x, self.nv, "x"), _dev3(y, self.nv, "y"), _stream()))
        return y

    def cloth_export_bell(self):
        """(cols (width, nv) int32, vals (9, width, nv) float64) on the device."""
        import torch
        w = ctypes.c_int32(0)
        self._check(lib().cloth_export_bell(self.h, ctypes.byref(w), None, None, _stream()))
        width = int(w.value)
        cols = torch.empty((width, self.nv), dtype=torch.int32, device="cuda")
        vals = torch.empty((9, width, self.nv), dtype=torch.float64, device="cuda")
        self._check(lib().cloth_export_bell(self.h, None, _ptr(cols), _ptr(vals), _stream()))
        return cols, vals

    def cloth_export_blocks(self, with_D=True, solver_blocks=False):
        import torch
        rowptr, colidx = self.pattern()
        vals = torch.empty((colidx.numel(), 3, 3), dtype=torch.float64, device="cuda")
        D = torch.empty((self.nv, 3, 3), dtype=torch.float64, device="cuda") if with_D else None
        self._check(lib().cloth_export_blocks(self.h, _ptr(vals), _ptr(D) if D is not None else None,
                                              int(solver_blocks), _stream()))
        return rowptr, colidx, vals, D

    def cloth_step(self, x, v, nsteps=1, dtype="f32", tol=1e-6, maxit=20000, warm=False, check_every=0,
                   inner_rho=0.0, max_sweeps=0, precond="jacobi", method="cg"):
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        o = solve_opts(tol, maxit, warm, check_every, inner_rho, max_sweeps, precond, method)
        infos = (PcSolveInfo * max(1, nsteps))()
        st = lib().cloth_step(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"), int(nsteps), dt,
                              ctypes.byref(o), infos, _stream())
        self._check(st)
        return [infos[k].as_dict() for k in range(nsteps)]

    # -- learned warm start --------------------------------------------------
    @staticmethod
    def ws_init_params(seed=0):
        """Seeded He-normal weights and zero biases in the flat layout; the last
        layer is scaled by 1e-2 so that an untrained network starts CG at the
        previous step's increment."""
        rng = np.random.default_rng(seed)
        parts = []
        for k, (a, b) in enumerate(WS_SHAPES):
            W = rng.normal(size=(a, b)) * np.sqrt(2.0 / a) * (1e-2 if k == len(WS_SHAPES) - 1 else 1.0)
            parts += [W.ravel(), np.zeros(b)]
        return np.concatenate(parts).astype(np.float32)

    def ws_set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == WS_PARAMS
        self._check(lib().pc_ws_set_params(self.h, a.ctypes.data_as(ctypes.c_void_p), WS_PARAMS))

    def ws_get_params(self):
        a = np.zeros(WS_PARAMS, dtype=np.float32)
        self._check(lib().pc_ws_get_params(self.h, a.ctypes.data_as(ctypes.c_void_p), WS_PARAMS))
        return a

    def ws_features(self, x, v, b, dv_prev):
        import torch
        out = torch.empty((self.nv, 32), dtype=torch.int16, device="cuda")
        self._check(lib().pc_ws_features(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"),
                                         _dev3(b, self.nv, "b"), _dev3(dv_prev, self.nv, "dv_prev"), _ptr(out),
                                         _stream()))
        return out

    def ws_predict(self, x, v, b, dv_prev):
        import torch
        out = torch.empty((self.nv, 3), dtype=torch.float64, device="cuda")
        self._check(lib().pc_ws_predict(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"),
                                        _dev3(b, self.nv, "b"), _dev3(dv_prev, self.nv, "dv_prev"), _ptr(out),
                                        _stream()))
        return out

    def ws_predict_noalloc(self, x, v, b, dv_prev, out=None):
        """pc_ws_predict without any allocation inside the library (the
        output tensor is the caller's)."""
        import torch
        if out is None:
            out = torch.empty((self.nv, 3), dtype=torch.float64, device="cuda")
        self._check(lib().pc_ws_predict_noalloc(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"),
                                                _dev3(b, self.nv, "b"), _dev3(dv_prev, self.nv, "dv_prev"),
                                                _dev3(out, self.nv, "out"), _stream()))
        return out

    def ws_start(self, x, v, b, dv_prev):
        """The learned CG start (previous increment plus a line-searched step
        along the network's correction) and its step."""
        import torch
        out = torch.empty((self.nv, 3), dtype=torch.float64, device="cuda")
        g = ctypes.c_double()
        self._check(lib().pc_ws_start(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"),
                                      _dev3(b, self.nv, "b"), _dev3(dv_prev, self.nv, "dv_prev"), _ptr(out),
                                      ctypes.byref(g), _stream()))
        return out, g.value

    def ws_gradient(self, x, v, b, dv_prev):
        g = np.zeros(WS_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(lib().pc_ws_gradient(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"),
                                         _dev3(b, self.nv, "b"), _dev3(dv_prev, self.nv, "dv_prev"),
                                         g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss), _stream()))
        return g, loss.value

    def ws_train_step(self, x, v, b, dv_prev, lr=1e-3, want_loss=True):
        loss = ctypes.c_double()
        self._check(lib().pc_ws_train_step(self.h, _dev3(x, self.nv, "x"), _dev3(v, self.nv, "v"),
                                           _dev3(b, self.nv, "b"), _dev3(dv_prev, self.nv, "dv_prev"),
                                           float(lr), ctypes.byref(loss) if want_loss else None, _stream()))
        return loss.value if want_loss else None

    def mfma_probe(self):
        out = np.zeros(1024, dtype=np.float32)
        self._check(lib().pc_mfma_probe(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape(4, 16, 16)

    def set_option(self, option, value):
        self._check(lib().pc_set_option(self.h, int(option), int(value)))

    def get_option(self, option):
        v = ctypes.c_int64()
        self._check(lib().pc_get_option(self.h, int(option), ctypes.byref(v)))
        return v.value

    def set_instances(self, vertex_begin):
        a = np.ascontiguousarray(vertex_begin, dtype=np.int32)
        self._check(lib().pc_set_instances(self.h, a.ctypes.data_as(ctypes.c_void_p), a.size - 1))
        self.ninst = a.size - 1

    def autotune(self, b, iters=64, cache=None, key=None, precond="jacobi"):
        """Pick the fastest launch schedule for the assembled system (see
        pc_autotune).  With a cache path and key, a previous choice is reused
        and new choices are stored (JSON)."""
        import json
        if cache and key and os.path.exists(cache):
            with open(cache) as fh:
                known = json.load(fh)
            if key in known:
                spb, rpb, chunk = known[key]["choice"]
                self.set_option(PC_OPT_SPMV_SLICES_PER_BLOCK, spb)
                self.set_option(PC_OPT_VECTOR_ROWS_PER_BLOCK, rpb)
                self.set_option(PC_OPT_GRAPH_CHUNK, chunk)
                return {"choice": [spb, rpb, chunk], "ms_per_iter": known[key]["ms_per_iter"], "cached": True}
        chosen = (ctypes.c_int64 * 3)()
        ms = ctypes.c_double()
        pre = PRECOND[precond] if isinstance(precond, str) else int(precond)
        self._check(lib().pc_autotune(self.h, _dev3(b, self.nv, "b"), int(iters), pre, chosen, ctypes.byref(ms),
                                      _stream()))
        res = {"choice": [chosen[0], chosen[1], chosen[2]], "ms_per_iter": ms.value, "cached": False}
        if cache and key:
            known = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    known = json.load(fh)
            known[key] = {"choice": res["choice"], "ms_per_iter": res["ms_per_iter"]}
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as fh:
                json.dump(known, fh, indent=1)
        return res

    def instance_info(self):
        n = getattr(self, "ninst", 1)
        arr = (PcSolveInfo * n)()
        self._check(lib().pc_get_instance_info(self.h, arr, n))
        return [arr[i].as_dict() for i in range(n)]

    def profile(self, every):
        self._check(lib().pc_profile(self.h, int(every)))

    def profile_read(self):
        out = (ctypes.c_double * 40)()
        self._check(lib().pc_profile_read(self.h, out))
        return {PROFILE_KINDS[k]: {"samples": int(out[5 * k]), "mean_ms": out[5 * k + 1], "min_ms": out[5 * k + 2],
                                   "max_ms": out[5 * k + 3], "median_ms": out[5 * k + 4]}
                for k in range(8) if out[5 * k] > 0}

    def check(self):
        self._check(lib().pc_check(self.h, _stream()))
