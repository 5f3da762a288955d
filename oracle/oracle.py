"""ctypes wrapper of the C oracle (``ipm_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

The oracle is a plain FP64 CPU implementation of the IPM hot path written
from the paper's equations (Sec. 3.1 eq:L, eq:dualIterationFunction,
eq:tauCrit, eq:momentIterationFunction, Algs. 1 and 2; App. B for the Euler
closure).  It shares no code with the GPU library.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_SRC = os.path.join(_HERE, "ipm_oracle.c")

EQ = {"burgers1d": 0, "euler1d": 1, "euler2d": 2}
ENT = {"quadratic": 0, "log_barrier": 1, "euler": 2}
FLUX = {"lf": 0, "rusanov": 1, "sg_analytic": 2}
BC = {"outflow": 0, "periodic": 1, "dirichlet": 2}
QUAD = {"gl": 0, "cc": 1, "cc_sparse": 2}
STATUS = {"newton": 1, "realizability": 2, "nonfinite": 4, "cholesky": 8, "linesearch": 16}


class Problem(C.Structure):
    _fields_ = [
        ("equation", C.c_int), ("entropy", C.c_int), ("flux", C.c_int),
        ("gamma", C.c_double), ("u_minus", C.c_double), ("u_plus", C.c_double),
        ("p", C.c_int), ("degree", C.c_int), ("quad_per_dim", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("bc", C.c_int * 4),
        ("cfl", C.c_double), ("t_end", C.c_double), ("tau", C.c_double),
        ("steady_eps", C.c_double),
        ("max_newton", C.c_int), ("one_shot", C.c_int),
        ("adapt", C.c_int), ("min_degree", C.c_int),
        ("delta_lo", C.c_double), ("delta_hi", C.c_double),
        ("n_retard", C.c_int), ("retard_degree", C.c_int * 16), ("retard_eps", C.c_double * 16),
        ("quad_rule", C.c_int),
    ]


class Info(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("dt", C.c_double), ("residual", C.c_double), ("amax", C.c_double),
        ("steps", C.c_longlong), ("newton_iters", C.c_longlong), ("cell_updates", C.c_longlong),
        ("max_iters", C.c_int), ("status", C.c_int), ("done", C.c_int),
        ("retard_stage", C.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force=False):
    """Compile the oracle with gcc (-O2, OpenMP over cells)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    return _SO


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = C.CDLL(_SO)
    d, i, P = C.c_double, C.c_int, C.POINTER
    dp, ip = P(C.c_double), P(C.c_int)
    lib.orc_num_basis.argtypes = [i, i]
    lib.orc_gauss_legendre.argtypes = [i, dp, dp]
    lib.orc_quadrature.argtypes = [i, i, dp, dp]
    lib.orc_clenshaw_curtis.argtypes = [i, dp, dp]
    lib.orc_quadrature_size.argtypes = [i, i, i]
    lib.orc_quadrature_rule.argtypes = [i, i, i, dp, dp]
    lib.orc_multi_indices.argtypes = [i, i, ip]
    lib.orc_basis_eval.argtypes = [i, i, i, dp, dp]
    lib.orc_basis_eval.restype = None
    lib.orc_indicator.argtypes = [i, i, i, dp, dp]
    lib.orc_indicator.restype = None
    lib.orc_select_degrees.argtypes = [i, i, i, i, i, dp, d, P(C.c_byte)]
    lib.orc_select_degrees.restype = None
    lib.orc_closure.argtypes = [i, i, d, d, d, dp, dp, dp, dp]
    lib.orc_entropy_grad.argtypes = [i, i, d, d, d, dp, dp]
    lib.orc_entropy.argtypes = [i, i, d, d, d, dp]
    lib.orc_entropy.restype = d
    lib.orc_create.argtypes = [P(Problem), P(C.c_byte), dp, dp]
    lib.orc_create.restype = C.c_void_p
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_destroy.restype = None
    lib.orc_sizes.argtypes = [C.c_void_p, ip, ip, ip, ip]
    lib.orc_sizes.restype = None
    lib.orc_step.argtypes = [C.c_void_p, i, P(Info)]
    lib.orc_get_info.argtypes = [C.c_void_p, P(Info)]
    lib.orc_get_info.restype = None
    for nm in ("orc_get_moments", "orc_set_moments", "orc_get_dual", "orc_set_dual"):
        getattr(lib, nm).argtypes = [C.c_void_p, dp]
        getattr(lib, nm).restype = None
    lib.orc_get_iters.argtypes = [C.c_void_p, ip]
    lib.orc_get_iters.restype = None
    lib.orc_get_degrees.argtypes = [C.c_void_p, P(C.c_byte)]
    lib.orc_get_degrees.restype = None
    lib.orc_get_nodal.argtypes = [C.c_void_p, dp]
    lib.orc_tables.argtypes = [C.c_void_p, dp, dp, dp]
    lib.orc_tables.restype = None
    lib.orc_dual_cost.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
    lib.orc_dual_solve.argtypes = [C.c_void_p, dp, dp, i, ip]
    lib.orc_moments_of_dual.argtypes = [C.c_void_p, dp, dp]
    lib.orc_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def num_basis(p, degree):
    return load().orc_num_basis(p, degree)


def gauss_legendre(n):
    x, w = np.zeros(n), np.zeros(n)
    load().orc_gauss_legendre(n, _ptr(x), _ptr(w))
    return x, w


def quadrature(p, qpd, rule="gl"):
    """Nodes [Q][p] and weights (sum 1) of a rule: gl / cc (qpd points per
    dimension) or cc_sparse (qpd = level)."""
    lib = load()
    Q = lib.orc_quadrature_size(QUAD[rule], p, qpd)
    nodes, w = np.zeros((Q, p)), np.zeros(Q)
    lib.orc_quadrature_rule(QUAD[rule], p, qpd, _ptr(nodes), _ptr(w))
    return nodes, w


def clenshaw_curtis(n):
    """n-point Clenshaw-Curtis rule on [-1, 1] (weights sum to 2)."""
    x, w = np.zeros(n), np.zeros(n)
    load().orc_clenshaw_curtis(n, _ptr(x), _ptr(w))
    return x, w


def multi_indices(p, degree):
    N = num_basis(p, degree)
    idx = np.zeros((N, p), dtype=np.int32)
    load().orc_multi_indices(p, degree, _ptr(idx, C.c_int))
    return idx


def basis_eval(p, degree, nodes):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, p)
    Phi = np.zeros((nodes.shape[0], num_basis(p, degree)))
    load().orc_basis_eval(p, degree, nodes.shape[0], _ptr(nodes), _ptr(Phi))
    return Phi


def indicator(p, L, qpd, u_nodes):
    """S_1..S_L of eq:errorIndicator for one scalar field at the Q nodes."""
    u = np.ascontiguousarray(u_nodes, dtype=np.float64).reshape(-1)
    S = np.zeros(L)
    load().orc_indicator(p, L, qpd, _ptr(u), _ptr(S))
    return S


def select_degrees(p, L, qpd, ic_nodal, delta_hi=1e-4):
    """Static per-cell total degree (1..L) from the indicator of the first
    conserved variable; ic_nodal [cells][Q][m]."""
    ic = np.ascontiguousarray(ic_nodal, dtype=np.float64)
    cells, Q, m = ic.shape
    out = np.zeros(cells, dtype=np.int8)
    load().orc_select_degrees(p, L, qpd, m, cells, _ptr(ic), float(delta_hi),
                              out.ctypes.data_as(C.POINTER(C.c_byte)))
    return out


def closure(entropy, m, Lam, gamma=1.4, um=0.0, up=1.0):
    """u_s(Lam), grad u_s(Lam), s_*(Lam) at one node; ok flag."""
    Lam = np.ascontiguousarray(Lam, dtype=np.float64)
    u, J, ss = np.zeros(m), np.zeros((m, m)), np.zeros(1)
    ok = load().orc_closure(ENT[entropy], m, gamma, um, up, _ptr(Lam), _ptr(u), _ptr(J), _ptr(ss))
    return u, J, ss[0], bool(ok)


def entropy_grad(entropy, m, u, gamma=1.4, um=0.0, up=1.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    Lam = np.zeros(m)
    ok = load().orc_entropy_grad(ENT[entropy], m, gamma, um, up, _ptr(u), _ptr(Lam))
    return Lam, bool(ok)


def entropy(entropy_name, m, u, gamma=1.4, um=0.0, up=1.0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return load().orc_entropy(ENT[entropy_name], m, gamma, um, up, _ptr(u))


def make_problem(spec):
    """Problem struct from a workload spec dict (see the workloads module)."""
    pb = Problem()
    pb.equation = EQ[spec["equation"]]
    pb.entropy = ENT[spec["entropy"]]
    pb.flux = FLUX[spec["flux"]]
    pb.gamma = spec.get("gamma", 1.4)
    pb.u_minus = spec.get("u_minus", 0.0)
    pb.u_plus = spec.get("u_plus", 1.0)
    pb.p = spec["p"]
    pb.degree = spec["degree"]
    pb.quad_per_dim = spec["quad_per_dim"]
    pb.nx = spec["nx"]
    pb.ny = spec.get("ny", 1)
    pb.x0, pb.x1 = spec["x0"], spec["x1"]
    pb.y0, pb.y1 = spec.get("y0", 0.0), spec.get("y1", 1.0)
    bcs = spec["bc"]
    for k in range(4):
        pb.bc[k] = BC[bcs[k]] if k < len(bcs) else 0
    pb.cfl = spec["cfl"]
    pb.t_end = spec.get("t_end", 0.0)
    pb.tau = spec.get("tau", 1e-10)
    pb.steady_eps = spec.get("steady_eps", 0.0)
    pb.max_newton = spec.get("max_newton", 100)
    pb.one_shot = int(spec.get("one_shot", 0))
    pb.quad_rule = QUAD[spec.get("quad_rule", "gl")]
    pb.adapt = int(spec.get("adapt", 0))
    pb.min_degree = spec.get("min_degree", 1)
    pb.delta_lo = spec.get("delta_lo", 0.0)
    pb.delta_hi = spec.get("delta_hi", 0.0)
    stages = spec.get("retard", ())  # [(max degree, residual tolerance), ...]
    pb.n_retard = len(stages)
    for k, (dg, eps) in enumerate(stages):
        pb.retard_degree[k] = dg
        pb.retard_eps[k] = eps
    return pb


class Oracle:
    """One IPM problem on the CPU.

    ``ic_nodal``: [cells][Q][m] initial state at the cell centres and the
    oracle's own quadrature nodes (``self.nodes``)."""

    def __init__(self, spec, ic_nodal=None, ic_fn=None, dirichlet_fn=None, cell_degree=None):
        lib = load()
        self.spec = dict(spec)
        self.pb = make_problem(spec)
        self.m = {0: 1, 1: 3, 2: 4}[self.pb.equation]
        self.N = num_basis(self.pb.p, self.pb.degree)
        self.nodes, self.w = quadrature(self.pb.p, self.pb.quad_per_dim,
                                        spec.get("quad_rule", "gl"))
        self.Q = self.nodes.shape[0]
        ny = self.pb.ny if self.pb.equation == 2 else 1
        self.cells = self.pb.nx * ny
        if ic_nodal is None:
            ic_nodal = ic_fn(self.nodes)
        ic = np.ascontiguousarray(ic_nodal, dtype=np.float64).reshape(self.cells, self.Q, self.m)
        dn = None
        if dirichlet_fn is not None:
            dn = np.ascontiguousarray(dirichlet_fn(self.nodes), dtype=np.float64).reshape(4, self.Q, self.m)
        cd = None
        if cell_degree is not None:
            cd = np.ascontiguousarray(cell_degree, dtype=np.int8)
            self._cd = cd
        self._h = lib.orc_create(C.byref(self.pb), _ptr(cd, C.c_byte) if cd is not None else None,
                                 _ptr(ic), _ptr(dn) if dn is not None else None)
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def step(self, max_steps=1):
        info = Info()
        self._lib.orc_step(self._h, int(max_steps), C.byref(info))
        return info.as_dict()

    def run(self, max_steps=10 ** 9):
        return self.step(max_steps)

    @property
    def info(self):
        info = Info()
        self._lib.orc_get_info(self._h, C.byref(info))
        return info.as_dict()

    def moments(self):
        out = np.zeros((self.cells, self.m, self.N))
        self._lib.orc_get_moments(self._h, _ptr(out))
        return out

    def set_moments(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._lib.orc_set_moments(self._h, _ptr(a))

    def dual(self):
        out = np.zeros((self.cells, self.m, self.N))
        self._lib.orc_get_dual(self._h, _ptr(out))
        return out

    def set_dual(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._lib.orc_set_dual(self._h, _ptr(a))

    def iters(self):
        out = np.zeros(self.cells, dtype=np.int32)
        self._lib.orc_get_iters(self._h, _ptr(out, C.c_int))
        return out

    def degrees(self):
        """Current total degree (refinement level) of every cell."""
        out = np.zeros(self.cells, dtype=np.int8)
        self._lib.orc_get_degrees(self._h, out.ctypes.data_as(C.POINTER(C.c_byte)))
        return out

    def nodal(self):
        out = np.zeros((self.cells, self.Q, self.m))
        self._lib.orc_get_nodal(self._h, _ptr(out))
        return out

    def tables(self):
        nodes = np.zeros((self.Q, self.pb.p))
        w = np.zeros(self.Q)
        Phi = np.zeros((self.Q, self.N))
        self._lib.orc_tables(self._h, _ptr(nodes), _ptr(w), _ptr(Phi))
        return nodes, w, Phi

    def dual_cost(self, lam, uhat, hessian=True):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        uhat = np.ascontiguousarray(uhat, dtype=np.float64)
        L = np.zeros(1)
        g = np.zeros((self.m, self.N))
        n = self.m * self.N
        H = np.zeros((n, n)) if hessian else None
        ok = self._lib.orc_dual_cost(self._h, _ptr(lam), _ptr(uhat), _ptr(L), _ptr(g),
                                     _ptr(H) if hessian else None)
        return L[0], g, H, bool(ok)

    def dual_solve(self, uhat, lam0, one_shot=False):
        uhat = np.ascontiguousarray(uhat, dtype=np.float64)
        lam = np.array(lam0, dtype=np.float64, order="C").reshape(self.m, self.N)
        it = C.c_int(0)
        st = self._lib.orc_dual_solve(self._h, _ptr(uhat), _ptr(lam), int(one_shot), C.byref(it))
        return lam, st, it.value

    def moments_of_dual(self, lam):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        u = np.zeros((self.m, self.N))
        ok = self._lib.orc_moments_of_dual(self._h, _ptr(lam), _ptr(u))
        return u, bool(ok)
