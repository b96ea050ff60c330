"""Python binding of libspock (MI355X / gfx950 SPOCK hot path).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch tensors on the current HIP device; the current
torch stream is passed to the library. Importing this package does not
require a GPU; calling a compute entry point does, and fails loudly if the
built library is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspock.so")

SPOCK_OK = 0
ERRORS = {-1: "SPOCK_EINVAL", -2: "SPOCK_ETREE", -3: "SPOCK_EPROB", -4: "SPOCK_EBOX",
          -5: "SPOCK_EFACTOR", -6: "SPOCK_EHIP", -7: "SPOCK_ENOMEM", -8: "SPOCK_EUNSUPPORTED",
          -9: "SPOCK_ETOOBIG"}
STATUS = {0: "converged", 1: "maxiter", 2: "numerical", 3: "rejected"}
FP64, FP32 = 0, 1
METHOD_CP, METHOD_SPOCK = 0, 1
AA_AUTO, AA_GRAM, AA_QR = 0, 1, 2

EXPORTED = [
    "spock_tree_create", "spock_tree_destroy", "spock_tree_shape", "spock_problem_factor",
    "spock_problem_destroy", "spock_problem_sizes", "spock_settings_default", "spock_solve",
    "spock_solve_batched", "spock_apply_L", "spock_apply_Lt", "spock_prox_f",
    "spock_prox_gstar", "spock_T", "spock_version", "spock_backward", "spock_profile_T",
    "spock_problem_mapping", "spock_T_noalloc", "spock_backward_batched",
]


class SpockError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {ERRORS.get(code, code)}")
        self.code = code


class _RiskData(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_void_p), ("nnu", ctypes.c_void_p), ("kpos", ctypes.c_void_p),
                ("E", ctypes.c_void_p), ("F", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class _ConstraintData(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int32), ("ncN", ctypes.c_int32),
                ("Gx", ctypes.c_void_p), ("Gu", ctypes.c_void_p), ("cmin", ctypes.c_void_p),
                ("cmax", ctypes.c_void_p), ("GN", ctypes.c_void_p), ("cNmin", ctypes.c_void_p),
                ("cNmax", ctypes.c_void_p)]


class _ProblemData(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("q", ctypes.c_void_p), ("r", ctypes.c_void_p), ("qN", ctypes.c_void_p),
                ("xmin", ctypes.c_void_p), ("xmax", ctypes.c_void_p),
                ("umin", ctypes.c_void_p), ("umax", ctypes.c_void_p),
                ("a_risk", ctypes.c_void_p), ("precision", ctypes.c_int32),
                ("alpha", ctypes.c_double),
                ("risk", ctypes.POINTER(_RiskData)), ("cons", ctypes.POINTER(_ConstraintData)),
                ("Qm", ctypes.c_void_p), ("Rm", ctypes.c_void_p), ("QNm", ctypes.c_void_p)]


def _risk_struct(risk, anc, keep):
    """Flattens per-node E, F, b (nonleaf nodes in breadth-first order) into
    the C layout; arrays are kept alive in `keep`."""
    nn = len(anc)
    nonleaf = sorted(set(int(a) for a in anc[1:]))
    ny = np.zeros(nn, dtype=np.int32)
    nnu = np.zeros(nn, dtype=np.int32)
    kpos = np.zeros(nn, dtype=np.int32)
    E, F, b = [], [], []
    for i in nonleaf:
        Ei = np.asarray(risk.E[i], dtype=np.float64)
        bi = np.asarray(risk.b[i], dtype=np.float64)
        Fi = np.asarray(risk.F[i], dtype=np.float64).reshape(len(bi), -1)
        ny[i], nnu[i], kpos[i] = len(bi), Fi.shape[1], int(risk.kpos[i])
        E.append(Ei.ravel())
        F.append(Fi.ravel())
        b.append(bi)
    arr = {"ny": ny, "nnu": nnu, "kpos": kpos, "E": np.ascontiguousarray(np.concatenate(E)),
           "F": np.ascontiguousarray(np.concatenate(F)) if sum(f.size for f in F) else np.zeros(1),
           "b": np.ascontiguousarray(np.concatenate(b))}
    keep.update({"risk_" + k: v for k, v in arr.items()})
    return _RiskData(**{k: v.ctypes.data for k, v in arr.items()})


def _cons_struct(cons, keep):
    arr = {k: np.ascontiguousarray(getattr(cons, k), dtype=np.float64)
           for k in ("Gx", "Gu", "cmin", "cmax", "GN", "cNmin", "cNmax")}
    keep.update({"cons_" + k: v for k, v in arr.items()})
    return _ConstraintData(nc=arr["Gx"].shape[1], ncN=arr["GN"].shape[1],
                           **{k: v.ctypes.data for k, v in arr.items()})


class Settings(ctypes.Structure):
    _fields_ = [("eps_abs", ctypes.c_double), ("eps_rel", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("method", ctypes.c_int32),
                ("m", ctypes.c_int32), ("max_ls", ctypes.c_int32),
                ("c0", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("beta", ctypes.c_double), ("sigma", ctypes.c_double),
                ("lam", ctypes.c_double), ("compute_nested", ctypes.c_int32),
                ("anderson", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("t_evals", ctypes.c_int32), ("n_k0", ctypes.c_int32), ("n_k1", ctypes.c_int32),
                ("n_k2", ctypes.c_int32), ("n_km", ctypes.c_int32),
                ("n_backtracks", ctypes.c_int32), ("xi0", ctypes.c_double),
                ("xi", ctypes.c_double), ("V_s0", ctypes.c_double),
                ("V_nested", ctypes.c_double), ("seconds", ctypes.c_double),
                ("mapping", ctypes.c_int32), ("flow_fallback", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status"] = STATUS.get(self.status, self.status)
        return d


_lib = None
# live handles, destroyed in order (problems, then trees) by an exit hook that
# runs before the interpreter and the HIP runtime shut down, so no handle is
# freed from a finaliser at an unknown point of the shutdown
_live_problems: "weakref.WeakSet" = None
_live_trees: "weakref.WeakSet" = None


def _track(obj, trees: bool):
    global _live_problems, _live_trees
    if _live_problems is None:
        _live_problems, _live_trees = weakref.WeakSet(), weakref.WeakSet()
        atexit.register(_destroy_all)
    (_live_trees if trees else _live_problems).add(obj)


def _destroy_all():
    for p in list(_live_problems or ()):
        p.close()
    for t in list(_live_trees or ()):
        t.close()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libspock.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.spock_tree_create.argtypes = [i32, vp, vp, ctypes.POINTER(vp)]
        L.spock_tree_destroy.argtypes = [vp]
        L.spock_tree_shape.argtypes = [vp, vp, vp, vp]
        L.spock_problem_factor.argtypes = [vp, ctypes.POINTER(_ProblemData), ctypes.POINTER(vp)]
        L.spock_problem_destroy.argtypes = [vp]
        L.spock_problem_sizes.argtypes = [vp, vp, vp, vp, vp]
        L.spock_problem_mapping.argtypes = [vp, vp, vp, vp]
        L.spock_settings_default.argtypes = [ctypes.POINTER(Settings)]
        L.spock_settings_default.restype = None
        L.spock_solve.argtypes = [vp, vp, ctypes.POINTER(Settings), vp, ctypes.POINTER(Info), vp]
        L.spock_solve_batched.argtypes = [i32, vp, vp, ctypes.POINTER(Settings), vp, vp, vp]
        L.spock_apply_L.argtypes = [vp, vp, vp, vp]
        L.spock_apply_Lt.argtypes = [vp, vp, vp, vp]
        L.spock_prox_f.argtypes = [vp, vp, vp, vp, vp]
        L.spock_prox_gstar.argtypes = [vp, vp, vp, vp]
        L.spock_T.argtypes = [vp, vp, vp, vp, vp, vp]
        L.spock_T_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
        L.spock_profile_T.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.spock_backward.argtypes = [vp, vp, vp, dbl, vp, vp, vp, vp, ctypes.POINTER(Settings),
                                     ctypes.POINTER(Info), vp]
        L.spock_backward_batched.argtypes = [vp, i32, vp, vp, dbl, vp, vp, vp, vp, ctypes.POINTER(Settings),
                                             vp, vp]
        L.spock_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc, where):
    if rc != SPOCK_OK:
        raise SpockError(rc, where)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def default_settings(**kw) -> Settings:
    s = Settings()
    lib().spock_settings_default(ctypes.byref(s))
    for k, v in kw.items():
        if k == "lambda":
            k = "lam"
        if k == "method" and isinstance(v, str):
            v = METHOD_CP if v.lower() == "cp" else METHOD_SPOCK
        if k == "anderson" and isinstance(v, str):
            v = {"auto": AA_AUTO, "gram": AA_GRAM, "qr": AA_QR}[v.lower()]
        setattr(s, k, v)
    return s


class Tree:
    """Scenario tree (breadth-first ancestors and node probabilities)."""

    def __init__(self, anc, prob):
        self._anc = np.ascontiguousarray(anc, dtype=np.int32)
        self._prob = np.ascontiguousarray(prob, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().spock_tree_create(len(self._anc), self._anc.ctypes.data,
                                       self._prob.ctypes.data, ctypes.byref(h)),
               "spock_tree_create")
        self.handle = h
        N, nl, nleaf = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        lib().spock_tree_shape(h, ctypes.byref(N), ctypes.byref(nl), ctypes.byref(nleaf))
        self.N, self.num_nonleaf, self.num_leaves = N.value, nl.value, nleaf.value
        self.num_nodes = len(self._anc)
        _track(self, trees=True)

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.spock_tree_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


class Problem:
    """Factored problem on the device (Alg. 1 in FP64, storage in `precision`)."""

    def __init__(self, tree: Tree, nx, nu, A, B, q, r, qN, xmin, xmax, umin, umax, a_risk,
                 precision=FP64, alpha=0.0, risk=None, cons=None, Qm=None, Rm=None, QNm=None):
        """Dense costs: Qm, Rm, QNm (num_nodes x n x n each, all three or
        none) replace the diagonals q, r, qN, which may then be None."""
        self.tree = tree
        arrs = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in
                dict(A=A, B=B, q=q, r=r, qN=qN, xmin=xmin, xmax=xmax, umin=umin,
                     umax=umax, a_risk=a_risk, Qm=Qm, Rm=Rm, QNm=QNm).items() if v is not None}
        self._keep = arrs
        self._risk, self._cons = risk, cons
        extra = {}
        if risk is not None:
            self._risk_c = _risk_struct(risk, tree._anc, extra)
        if cons is not None:
            self._cons_c = _cons_struct(cons, extra)
        self._keep_general = extra
        d = _ProblemData(nx=nx, nu=nu, precision=precision, alpha=alpha,
                         risk=ctypes.pointer(self._risk_c) if risk is not None else None,
                         cons=ctypes.pointer(self._cons_c) if cons is not None else None,
                         **{k: v.ctypes.data for k, v in arrs.items()})
        h = ctypes.c_void_p()
        _check(lib().spock_problem_factor(tree.handle, ctypes.byref(d), ctypes.byref(h)),
               "spock_problem_factor")
        self.handle = h
        self.nx, self.nu, self.precision = nx, nu, precision
        nz, ne, al, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        lib().spock_problem_sizes(h, ctypes.byref(nz), ctypes.byref(ne), ctypes.byref(al),
                                  ctypes.byref(nl))
        self.n_z, self.n_eta, self.alpha, self.norm_L = nz.value, ne.value, al.value, nl.value
        self.n_v = self.n_z + self.n_eta
        _track(self, trees=False)

    @classmethod
    def from_instance(cls, inst, precision=FP64, alpha=0.0, tree=None):
        tree = tree or Tree(inst.anc, inst.prob)
        return cls(tree, inst.nx, inst.nu, inst.A, inst.B, inst.q, inst.r, inst.qN, inst.xmin,
                   inst.xmax, inst.umin, inst.umax, inst.a_risk, precision, alpha,
                   getattr(inst, "risk", None), getattr(inst, "cons", None),
                   getattr(inst, "Qm", None), getattr(inst, "Rm", None), getattr(inst, "QNm", None))

    def mapping(self) -> dict:
        """Mapping the next evaluation of T uses, the dataflow grid, and
        whether the dataflow form was given up for this problem."""
        m, g, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().spock_problem_mapping(self.handle, ctypes.byref(m), ctypes.byref(g), ctypes.byref(f)),
               "spock_problem_mapping")
        return {"mapping": m.value, "flow_grid": g.value, "flow_failed": bool(f.value)}

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.spock_problem_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()

    def refactor(self, q=None, r=None, qN=None, x_box=None, precision=None, alpha=0.0) -> "Problem":
        """A new problem on the same tree with some cost diagonals replaced
        (Alg. 1 runs again)."""
        k = dict(self._keep)
        for name, val in (("q", q), ("r", r), ("qN", qN)):
            if val is not None:
                k[name] = np.asarray(val, dtype=np.float64)
        if x_box is not None:
            k["xmin"], k["xmax"] = (np.asarray(b, dtype=np.float64) for b in x_box)
        return Problem(self.tree, self.nx, self.nu, k["A"], k["B"], k.get("q"), k.get("r"), k.get("qN"),
                       k["xmin"], k["xmax"], k["umin"], k["umax"], k["a_risk"],
                       self.precision if precision is None else precision, alpha, self._risk, self._cons,
                       k.get("Qm"), k.get("Rm"), k.get("QNm"))

    @property
    def q(self) -> np.ndarray:
        return self._keep.get("q")

    # ---- entry points
    def solve(self, x0, v, settings: Settings | None = None) -> dict:
        s = settings or default_settings()
        info = Info()
        _check(lib().spock_solve(self.handle, _ptr(x0), ctypes.byref(s), _ptr(v),
                                 ctypes.byref(info), _stream()), "spock_solve")
        return info.as_dict()

    def apply_L(self, z, eta):
        _check(lib().spock_apply_L(self.handle, _ptr(z), _ptr(eta), _stream()), "spock_apply_L")

    def apply_Lt(self, eta, z):
        _check(lib().spock_apply_Lt(self.handle, _ptr(eta), _ptr(z), _stream()), "spock_apply_Lt")

    def prox_f(self, zin, x0, zout):
        _check(lib().spock_prox_f(self.handle, _ptr(zin), _ptr(x0), _ptr(zout), _stream()),
               "spock_prox_f")

    def prox_gstar(self, w, out):
        _check(lib().spock_prox_gstar(self.handle, _ptr(w), _ptr(out), _stream()),
               "spock_prox_gstar")

    def backward(self, v_star, x0, gV=1.0, gu0=None, want_q=True, settings: Settings | None = None):
        """Gradients of gV * V* + gu0 . u0 with respect to x0, diag(Q) and
        diag(Q_N) at the solution v_star; returns (grad_x0, grad_q, grad_qN,
        info) as FP64 device tensors."""
        import torch
        s = settings or default_settings(eps_abs=1e-12, max_iters=200000)
        gx = torch.zeros(self.nx, dtype=torch.float64, device=x0.device)
        gq = torch.zeros((self.tree.num_nodes, self.nx), dtype=torch.float64, device=x0.device) if want_q else None
        gqN = torch.zeros_like(gq) if want_q else None
        info = Info()
        _check(lib().spock_backward(self.handle, _ptr(v_star), _ptr(x0), float(gV),
                                    _ptr(gu0) if gu0 is not None else None, _ptr(gx),
                                    _ptr(gq) if want_q else None, _ptr(gqN) if want_q else None,
                                    ctypes.byref(s), ctypes.byref(info), _stream()),
               "spock_backward")
        return gx, gq, gqN, info.as_dict()

    def profile_T(self, v, x0, Tv, reps=20):
        """Mean microseconds per phase of T over reps evaluations (HIP events
        on the current stream): pre, sweeps, post, reduce, total."""
        us = np.zeros(5)
        _check(lib().spock_profile_T(self.handle, _ptr(v), _ptr(x0), _ptr(Tv), int(reps),
                                     ctypes.c_void_p(us.ctypes.data), _stream()), "spock_profile_T")
        return dict(zip(("pre", "sweeps", "post", "reduce", "total"), us.tolist()))

    def T_noalloc(self, v, x0, Tv, want_stats=True):
        """spock_T_noalloc: T(v) with no device allocation (fixed scratch)."""
        st = np.zeros(6) if want_stats else None
        _check(lib().spock_T_noalloc(self.handle, _ptr(v), _ptr(x0), _ptr(Tv),
                                     ctypes.c_void_p(st.ctypes.data) if want_stats else None, _stream()),
               "spock_T_noalloc")
        if st is None:
            return None
        return dict(xi_p=st[0], xi_d=st[1], omega2=st[2], rz2=st[3], re2=st[4], cross=st[5])

    def T(self, v, x0, Tv, want_stats=True):
        st = np.zeros(6) if want_stats else None
        _check(lib().spock_T(self.handle, _ptr(v), _ptr(x0), _ptr(Tv),
                             ctypes.c_void_p(st.ctypes.data) if want_stats else None, _stream()),
               "spock_T")
        if st is None:
            return None
        return dict(xi_p=st[0], xi_d=st[1], omega2=st[2], rz2=st[3], re2=st[4], cross=st[5])


def solve_batched(problems, x0s, vs, settings: Settings | None = None):
    s = settings or default_settings()
    B = len(problems)
    ph = (ctypes.c_void_p * B)(*[p.handle.value for p in problems])
    xp = (ctypes.c_void_p * B)(*[x.data_ptr() for x in x0s])
    vp = (ctypes.c_void_p * B)(*[v.data_ptr() for v in vs])
    infos = (Info * B)()
    _check(lib().spock_solve_batched(B, ph, xp, ctypes.byref(s), vp, infos, _stream()),
           "spock_solve_batched")
    return [i.as_dict() for i in infos]


def backward_batched(problem, v_stars, x0s, gV=1.0, gu0s=None, want_q=True, settings: Settings | None = None):
    """spock_backward_batched: the gradients of spock_backward for the
    instances (v_stars[b], x0s[b]) of one problem at once; returns a list of
    (grad_x0, grad_q, grad_qN, info) per instance (FP64 device tensors)."""
    import torch
    s = settings or default_settings(eps_abs=1e-12, max_iters=200000)
    B = len(v_stars)
    dev = x0s[0].device
    gx = [torch.zeros(problem.nx, dtype=torch.float64, device=dev) for _ in range(B)]
    shape = (problem.tree.num_nodes, problem.nx)
    gq = [torch.zeros(shape, dtype=torch.float64, device=dev) for _ in range(B)] if want_q else None
    gqN = [torch.zeros(shape, dtype=torch.float64, device=dev) for _ in range(B)] if want_q else None
    arr = lambda ts: (ctypes.c_void_p * B)(*[t.data_ptr() if t is not None else None for t in ts])
    infos = (Info * B)()
    _check(lib().spock_backward_batched(problem.handle, B, arr(v_stars), arr(x0s), float(gV),
                                        arr(gu0s) if gu0s is not None else None, arr(gx),
                                        arr(gq) if want_q else None, arr(gqN) if want_q else None,
                                        ctypes.byref(s), infos, _stream()), "spock_backward_batched")
    return [(gx[b], gq[b] if want_q else None, gqN[b] if want_q else None, infos[b].as_dict()) for b in range(B)]


def version() -> str:
    return lib().spock_version().decode()
