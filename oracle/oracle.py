"""FP64 CPU oracle, Python side.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module; the product library never does.  It wraps the plain C oracle in
``pcloth_oracle.c`` (built with gcc, no HIP) and adds NumPy helpers for tiny
meshes.  Arrays on this side are (nv, 3) row-major float64.

Paper references: Sec. 2.5 (Eq. 1-3: backward Euler, the linear system
(M - dt^2 J) dv = dt f(u + dt v) and its PCG solve), Sec. 3.2.2 (the block
sparse matrix built from per-element contributions each step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcloth_oracle.c")
_LIB = os.path.join(_HERE, "libpcloth_oracle.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class OrParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("mu", ctypes.c_double), ("lam", ctypes.c_double),
                ("kb", ctypes.c_double), ("beta", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("rhs_mode", ctypes.c_int), ("hess_mode", ctypes.c_int)]


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_stretch_energy.restype = ctypes.c_double
        L.or_bend_energy.restype = ctypes.c_double
        L.or_hinge_angle.restype = ctypes.c_double
        L.or_contact_energy.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def num_threads() -> int:
    return int(lib().or_num_threads())


# ------------------------------------------------------------------ elements
def rest_triangles(X, tris):
    X, tris = _f64(X), _i32(tris)
    nt = tris.shape[0]
    B = np.zeros((nt, 4))
    A0 = np.zeros(nt)
    st = lib().or_rest_triangles(nt, _p(X, _f64p), _p(tris, _i32p), _p(B, _f64p), _p(A0, _f64p))
    if st != 0:
        raise ValueError(f"degenerate rest triangle {-1 - st}")
    return B, A0


def stretch_energy(x9, B, A0, mu, lam):
    x9, B = _f64(x9), _f64(B)
    return lib().or_stretch_energy(_p(x9, _f64p), _p(B, _f64p), ctypes.c_double(A0),
                                   ctypes.c_double(mu), ctypes.c_double(lam))


def stretch_force(x9, B, A0, mu, lam):
    x9, B = _f64(x9), _f64(B)
    f = np.zeros(9)
    lib().or_stretch_force(_p(x9, _f64p), _p(B, _f64p), ctypes.c_double(A0), ctypes.c_double(mu),
                           ctypes.c_double(lam), _p(f, _f64p))
    return f


def stretch_K(x9, B, A0, mu, lam, exact=False):
    x9, B = _f64(x9), _f64(B)
    K = np.zeros((9, 9))
    lib().or_stretch_K(_p(x9, _f64p), _p(B, _f64p), ctypes.c_double(A0), ctypes.c_double(mu),
                       ctypes.c_double(lam), int(exact), _p(K, _f64p))
    return K


def hinge_angle(x12):
    x12 = _f64(x12)
    return lib().or_hinge_angle(_p(x12, _f64p))


def hinge_grad(x12):
    x12 = _f64(x12)
    g = np.zeros(12)
    lib().or_hinge_grad(_p(x12, _f64p), _p(g, _f64p))
    return g


def bend_energy(x12, ch, tbar, kb):
    x12 = _f64(x12)
    return lib().or_bend_energy(_p(x12, _f64p), ctypes.c_double(ch), ctypes.c_double(tbar),
                                ctypes.c_double(kb))


def bend_force(x12, ch, tbar, kb):
    x12 = _f64(x12)
    f = np.zeros(12)
    lib().or_bend_force(_p(x12, _f64p), ctypes.c_double(ch), ctypes.c_double(tbar),
                        ctypes.c_double(kb), _p(f, _f64p))
    return f


def bend_K(x12, ch, tbar, kb, exact=False):
    x12 = _f64(x12)
    K = np.zeros((12, 12))
    lib().or_bend_K(_p(x12, _f64p), ctypes.c_double(ch), ctypes.c_double(tbar), ctypes.c_double(kb),
                    int(exact), _p(K, _f64p))
    return K


def contact_energy(x12, c, n, eta, kc):
    x12, c, n = _f64(x12), _f64(c), _f64(n)
    return lib().or_contact_energy(_p(x12, _f64p), _p(c, _f64p), _p(n, _f64p), ctypes.c_double(eta),
                                   ctypes.c_double(kc))


def contact_force(x12, c, n, eta, kc):
    x12, c, n = _f64(x12), _f64(c), _f64(n)
    f = np.zeros(12)
    lib().or_contact_force(_p(x12, _f64p), _p(c, _f64p), _p(n, _f64p), ctypes.c_double(eta), ctypes.c_double(kc),
                           _p(f, _f64p))
    return f


def contact_K(x12, c, n, eta, kc):
    x12, c, n = _f64(x12), _f64(c), _f64(n)
    K = np.zeros((12, 12))
    lib().or_contact_K(_p(x12, _f64p), _p(c, _f64p), _p(n, _f64p), ctypes.c_double(eta), ctypes.c_double(kc),
                       _p(K, _f64p))
    return K


@dataclass
class Contacts:
    """Proximity pairs of one step (the collision query's output): vertices
    (nc, 4) int32, weights (nc, 4) summing to zero per pair, unit normals
    (nc, 3), thickness eta and stiffness kc."""
    verts: np.ndarray
    weights: np.ndarray
    normals: np.ndarray
    eta: float
    kc: float

    @property
    def n(self):
        return int(self.verts.shape[0])


# ------------------------------------------------------------------ topology
def build_hinges(nv, tris):
    tris = _i32(tris)
    nt = tris.shape[0]
    cap = 3 * nt // 2 + 1
    hinges = np.zeros((cap, 4), dtype=np.int32)
    H = lib().or_build_hinges(int(nv), nt, _p(tris, _i32p), _p(hinges, _i32p), cap)
    if H < 0:
        raise ValueError({-1: "non-manifold edge", -2: "inconsistent orientation",
                          -3: "hinge capacity"}[H])
    return hinges[:H].copy()


def rest_hinges(X, hinges):
    X, hinges = _f64(X), _i32(hinges)
    H = hinges.shape[0]
    ch = np.zeros(H)
    tb = np.zeros(H)
    lib().or_rest_hinges(_p(X, _f64p), H, _p(hinges, _i32p), _p(ch, _f64p), _p(tb, _f64p))
    return ch, tb


def pattern(nv, tris, hinges, cverts=None):
    tris, hinges = _i32(tris), _i32(hinges)
    cverts = _i32(np.zeros((0, 4)) if cverts is None else cverts)
    nc = cverts.shape[0]
    cap = 9 * tris.shape[0] + 16 * hinges.shape[0] + 16 * nc + nv
    rowptr = np.zeros(nv + 1, dtype=np.int32)
    colidx = np.zeros(cap, dtype=np.int32)
    nnzb = lib().or_pattern2(int(nv), tris.shape[0], _p(tris, _i32p), hinges.shape[0],
                             _p(hinges, _i32p), nc, _p(cverts, _i32p), _p(rowptr, _i32p), _p(colidx, _i32p), cap)
    if nnzb < 0:
        raise RuntimeError("pattern capacity")
    return rowptr, colidx[:nnzb].copy()


# ------------------------------------------------------------------ problem
@dataclass
class Material:
    mu: float = 1000.0
    lam: float = 500.0
    kb: float = 1e-5
    beta: float = 0.0
    gravity: tuple = (0.0, 0.0, -9.81)
    rhs_mode: int = 1
    hess_mode: int = 0


@dataclass
class Assembled:
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray   # (nnzb, 3, 3)
    b: np.ndarray      # (nv, 3)
    diag: np.ndarray   # (nv, 3)
    D: np.ndarray      # (nv, 3, 3)

    def dense(self):
        nv = self.rowptr.size - 1
        A = np.zeros((3 * nv, 3 * nv))
        for i in range(nv):
            for p in range(self.rowptr[i], self.rowptr[i + 1]):
                j = self.colidx[p]
                A[3 * i:3 * i + 3, 3 * j:3 * j + 3] = self.vals[p]
        return A


class Problem:
    """Static data of one cloth (topology and rest shape) plus the oracle's
    step operations on it."""

    def __init__(self, rest, tris, mass, pinned, h, mat: Material | None = None):
        self.mat = mat or Material()
        self.rest = _f64(rest)
        self.tris = _i32(tris)
        self.mass = _f64(mass)
        self.pinned = np.ascontiguousarray(pinned, dtype=np.uint8)
        self.h = float(h)
        self.nv = self.rest.shape[0]
        self.nt = self.tris.shape[0]
        self.B, self.A0 = rest_triangles(self.rest, self.tris)
        self.hinges = build_hinges(self.nv, self.tris)
        self.ch, self.tbar = rest_hinges(self.rest, self.hinges)
        self.contacts = None
        self.rowptr, self.colidx = pattern(self.nv, self.tris, self.hinges)

    def set_contacts(self, contacts: "Contacts | None"):
        """Proximity pairs for the following assemblies; the pattern gains
        every pair of their vertices (None removes them)."""
        if contacts is not None:
            contacts = Contacts(_i32(contacts.verts).reshape(-1, 4), _f64(contacts.weights).reshape(-1, 4),
                                _f64(contacts.normals).reshape(-1, 3), float(contacts.eta), float(contacts.kc))
        self.contacts = contacts
        cv = contacts.verts if contacts is not None else None
        self.rowptr, self.colidx = pattern(self.nv, self.tris, self.hinges, cv)

    @classmethod
    def from_cloth(cls, c, mat: Material | None = None):
        return cls(c.rest, c.tris, c.mass, c.pinned, c.h, mat)

    @property
    def H(self):
        return self.hinges.shape[0]

    @property
    def nnzb(self):
        return int(self.rowptr[-1])

    def params(self):
        m = self.mat
        P = OrParams()
        P.h, P.mu, P.lam, P.kb, P.beta = self.h, m.mu, m.lam, m.kb, m.beta
        for a in range(3):
            P.g[a] = m.gravity[a]
        P.rhs_mode, P.hess_mode = m.rhs_mode, m.hess_mode
        return P

    def assemble(self, x, v) -> Assembled:
        x, v = _f64(x), _f64(v)
        nnzb = self.nnzb
        vals = np.zeros((nnzb, 3, 3))
        b = np.zeros((self.nv, 3))
        diag = np.zeros((self.nv, 3))
        D = np.zeros((self.nv, 3, 3))
        P = self.params()
        C = self.contacts
        nc = C.n if C is not None else 0
        cv = C.verts if nc else np.zeros((1, 4), np.int32)
        cw = C.weights if nc else np.zeros((1, 4))
        cn = C.normals if nc else np.zeros((1, 3))
        st = lib().or_assemble2(self.nv, self.nt, _p(self.tris, _i32p), _p(self.B, _f64p),
                               _p(self.A0, _f64p), self.H, _p(self.hinges, _i32p),
                               _p(self.ch, _f64p), _p(self.tbar, _f64p), nc, _p(cv, _i32p), _p(cw, _f64p),
                               _p(cn, _f64p), ctypes.c_double(C.eta if nc else 0.0),
                               ctypes.c_double(C.kc if nc else 0.0), _p(self.mass, _f64p),
                               _p(self.pinned, _u8p), ctypes.byref(P), _p(x, _f64p), _p(v, _f64p),
                               _p(self.rowptr, _i32p), _p(self.colidx, _i32p), _p(vals, _f64p),
                               _p(b, _f64p), _p(diag, _f64p), _p(D, _f64p))
        if st != 0:
            raise RuntimeError("assembly: pattern mismatch")
        return Assembled(self.rowptr, self.colidx, vals, b, diag, D)

    def spmv(self, A: Assembled, x):
        x = _f64(x)
        y = np.zeros_like(x)
        vals = _f64(A.vals)
        lib().or_spmv(self.nv, _p(A.rowptr, _i32p), _p(A.colidx, _i32p), _p(vals, _f64p),
                      _p(x, _f64p), _p(y, _f64p))
        return y

    def pcg(self, A: Assembled, x0=None, tol=1e-8, maxit=20000, precond="jacobi", method="cg"):
        """Preconditioned CG: precond "jacobi" (diag(A)) or "block" (the 3x3
        diagonal blocks of A); method "cg" (the textbook recurrences) or
        "chronopoulos-gear" (one fused reduction per iteration)."""
        x = np.zeros((self.nv, 3)) if x0 is None else _f64(x0).copy()
        out = np.zeros(4)
        vals = _f64(A.vals)
        pre = {"jacobi": 0, "block": 1}[precond]
        fn = {"cg": lib().or_pcg2, "chronopoulos-gear": lib().or_pcg_cg}[method]
        st = fn(self.nv, _p(A.rowptr, _i32p), _p(A.colidx, _i32p), _p(vals, _f64p),
                _p(A.b, _f64p), _p(A.diag, _f64p), _p(x, _f64p), ctypes.c_double(tol),
                int(maxit), int(pre), _p(out, _f64p))
        return x, {"converged": st == 0, "iters": int(out[0]), "rel_res_recursive": out[1],
                   "rel_res_true": out[2], "breakdown": bool(out[3])}

    def pcg_fixed(self, A: Assembled, iters: int):
        x = np.zeros((self.nv, 3))
        out = np.zeros(3)
        vals = _f64(A.vals)
        lib().or_pcg_fixed(self.nv, _p(A.rowptr, _i32p), _p(A.colidx, _i32p), _p(vals, _f64p),
                           _p(A.b, _f64p), _p(A.diag, _f64p), _p(x, _f64p), int(iters),
                           _p(out, _f64p))
        return x, out

    def update(self, x, v, dv):
        x, v = _f64(x).copy(), _f64(v).copy()
        dv = _f64(dv)
        lib().or_update(self.nv, _p(self.pinned, _u8p), ctypes.c_double(self.h), _p(dv, _f64p),
                        _p(x, _f64p), _p(v, _f64p))
        return x, v

    def step(self, x, v, tol=1e-6, maxit=20000, x0=None):
        A = self.assemble(x, v)
        dv, info = self.pcg(A, x0=x0, tol=tol, maxit=maxit)
        x1, v1 = self.update(x, v, dv)
        return x1, v1, dv, info

    def residual(self, A: Assembled, dv):
        """||b - A dv|| / ||b|| through the oracle's FP64 matrix."""
        r = A.b - self.spmv(A, dv)
        nb = np.linalg.norm(A.b)
        return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))
