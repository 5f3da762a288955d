"""ctypes binding of libipm (include/ipm.h): argument marshalling only.

Every step of the method runs in the HIP kernels of ``libipm.so``; this
module converts Python specs and NumPy / torch buffers to the C structures
and pointers the ABI takes.  It fails loudly when the library is missing.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipm.so")

EQ = {"burgers1d": 0, "euler1d": 1, "euler2d": 2}
ENT = {"quadratic": 0, "log_barrier": 1, "euler": 2}
FLUX = {"lf": 0, "rusanov": 1, "sg_analytic": 2}
BC = {"outflow": 0, "periodic": 1, "dirichlet": 2}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
QUAD = {"gl": 0, "cc": 1, "cc_sparse": 2}
STATUS = {0: "ok", -1: "arg", -2: "state", -3: "nomem", -4: "realizability", -5: "newton",
          -6: "nonfinite", -7: "device", -8: "busy"}


class IpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libipm error %d (%s): %s" % (code, STATUS.get(code, "?"), msg))
        self.code = code


class Config(C.Structure):
    _fields_ = [("device", C.c_int), ("hip_stream", C.c_void_p),
                ("hbm_budget_bytes", C.c_size_t), ("max_problems", C.c_int)]


class Problem(C.Structure):
    _fields_ = [
        ("equation", C.c_int), ("entropy", C.c_int), ("flux", C.c_int),
        ("gamma", C.c_double), ("u_minus", C.c_double), ("u_plus", C.c_double),
        ("p", C.c_int), ("degree", C.c_int), ("cell_degree", C.POINTER(C.c_int8)),
        ("quad_per_dim", C.c_int),
        ("cfl", C.c_double), ("t_end", C.c_double), ("tau", C.c_double), ("steady_eps", C.c_double),
        ("max_newton", C.c_int), ("one_shot", C.c_int), ("precision", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("bc", C.c_int * 4),
        ("ic_nodal", C.POINTER(C.c_double)), ("ic_moments", C.POINTER(C.c_double)),
        ("ic_dual", C.POINTER(C.c_double)), ("dirichlet", C.POINTER(C.c_double)),
        ("adapt", C.c_int), ("min_degree", C.c_int),
        ("delta_lo", C.c_double), ("delta_hi", C.c_double),
        ("n_retard", C.c_int), ("retard_degree", C.POINTER(C.c_int)),
        ("retard_eps", C.POINTER(C.c_double)), ("quad_rule", C.c_int),
        ("hessian_reuse", C.c_int),
        ("reuse_theta", C.c_double),
    ]


class StepInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("done", C.c_int), ("steps", C.c_longlong),
                ("t", C.c_double), ("dt", C.c_double), ("residual", C.c_double),
                ("amax", C.c_double), ("newton_iters", C.c_longlong),
                ("cell_updates", C.c_longlong), ("max_iters", C.c_int),
                ("retard_stage", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LaunchTime(C.Structure):
    _fields_ = [("m", C.c_int), ("lanes", C.c_int), ("workgroup", C.c_int), ("variant", C.c_int),
                ("threads", C.c_int), ("launches", C.c_longlong), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ClassStat(C.Structure):
    _fields_ = [("size_class", C.c_int), ("workgroup", C.c_int), ("lanes", C.c_int),
                ("variant", C.c_int), ("n_min", C.c_int), ("n_max", C.c_int),
                ("cells", C.c_longlong), ("listed", C.c_longlong),
                ("iterations", C.c_longlong), ("fresh", C.c_longlong),
                ("evaluations", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("problem", C.c_void_p), ("arrival_s", C.c_double),
                ("moments_out", C.POINTER(C.c_double)), ("moments_len", C.c_size_t),
                ("admitted_s", C.c_double), ("finished_s", C.c_double), ("steps", C.c_longlong),
                ("status", C.c_int), ("reserved", C.c_int)]


EXPORTS = ["ipm_create", "ipm_destroy", "ipm_quadrature", "ipm_basis_size", "ipm_basis_table",
           "ipm_set_problem", "ipm_step", "ipm_query", "ipm_moments", "ipm_dual",
           "ipm_problem_sizes", "ipm_problem_footprint", "ipm_release", "ipm_kernel_timing",
           "ipm_select_degrees", "ipm_serve", "ipm_autotune", "ipm_cell_degrees",
           "ipm_quadrature_size", "ipm_quadrature_rule", "ipm_last_error", "ipm_step_static",
           "ipm_launch_times", "ipm_class_stats"]

_lib = None


def load(path=None):
    """Load libipm.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError("libipm.so not built (%s); run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    P, dp, ip, vp = C.POINTER, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
    lib.ipm_create.argtypes = [P(Config), P(vp)]
    lib.ipm_destroy.argtypes = [vp]
    lib.ipm_quadrature.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int]
    lib.ipm_basis_size.argtypes = [C.c_int, C.c_int]
    lib.ipm_basis_table.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int]
    lib.ipm_set_problem.argtypes = [vp, P(Problem), ip]
    lib.ipm_step.argtypes = [vp, C.c_int, ip, C.c_int, P(StepInfo)]
    lib.ipm_step_static.argtypes = [vp, C.c_int, ip, C.c_int, P(StepInfo)]
    lib.ipm_launch_times.argtypes = [vp, P(LaunchTime), C.c_int, ip]
    lib.ipm_class_stats.argtypes = [vp, C.c_int, P(ClassStat), C.c_int, ip]
    lib.ipm_query.argtypes = [vp, C.c_int, P(StepInfo)]
    lib.ipm_moments.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
    lib.ipm_dual.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
    lib.ipm_problem_sizes.argtypes = [vp, C.c_int, ip, ip, ip, ip]
    lib.ipm_problem_footprint.argtypes = [P(Problem)]
    lib.ipm_problem_footprint.restype = C.c_size_t
    lib.ipm_release.argtypes = [vp, C.c_int]
    lib.ipm_kernel_timing.argtypes = [vp, C.c_int, dp, dp, P(C.c_longlong)]
    lib.ipm_autotune.argtypes = [vp, C.c_int, ip, C.c_int, ip]
    lib.ipm_serve.argtypes = [vp, C.c_int, P(Request), C.c_int, C.c_int]
    lib.ipm_select_degrees.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_double,
                                       P(C.c_int8)]
    lib.ipm_cell_degrees.argtypes = [vp, C.c_int, P(C.c_int8), C.c_size_t]
    lib.ipm_quadrature_size.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.ipm_quadrature_rule.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int]
    lib.ipm_last_error.argtypes = [vp]
    lib.ipm_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def quadrature(p, qpd, rule="gl"):
    """Nodes [Q][p] and weights of the problem's rule (``rule``: gl, cc or
    cc_sparse; qpd = points per dimension or the sparse level)."""
    lib = load()
    Q = lib.ipm_quadrature_size(QUAD[rule], p, qpd)
    nodes, w = np.zeros((max(Q, 1), p)), np.zeros(max(Q, 1))
    st = lib.ipm_quadrature_rule(QUAD[rule], p, qpd, _dptr(nodes), _dptr(w), Q)
    if st != 0:
        raise IpmError(st, lib.ipm_last_error(None).decode())
    return nodes, w


def basis_table(p, degree, qpd):
    lib = load()
    Q, N = qpd ** p, lib.ipm_basis_size(p, degree)
    Phi = np.zeros((Q, N))
    st = lib.ipm_basis_table(p, degree, qpd, _dptr(Phi), Q * N)
    if st != 0:
        raise IpmError(st, lib.ipm_last_error(None).decode())
    return Phi


def select_degrees(p, max_degree, qpd, ic_nodal, delta_hi=1e-4):
    """Per-cell total degree 1..max_degree from the smoothness indicator of
    the first conserved variable (ipm_select_degrees); ic_nodal [cells][Q][m]."""
    lib = load()
    ic = np.ascontiguousarray(ic_nodal, dtype=np.float64)
    cells, _, m = ic.shape
    out = np.zeros(cells, dtype=np.int8)
    st = lib.ipm_select_degrees(p, max_degree, qpd, m, cells, _dptr(ic), float(delta_hi),
                                out.ctypes.data_as(C.POINTER(C.c_int8)))
    if st != 0:
        raise IpmError(st, lib.ipm_last_error(None).decode())
    return out


def problem_struct(spec, keep):
    """Fill the C problem struct from a workload spec; arrays go in keep."""
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
    pb.cfl = spec["cfl"]
    pb.t_end = spec.get("t_end", 0.0)
    pb.tau = spec.get("tau", 1e-10)
    pb.steady_eps = spec.get("steady_eps", 0.0)
    pb.max_newton = spec.get("max_newton", 100)
    pb.one_shot = int(spec.get("one_shot", 0))
    pb.precision = PREC[spec.get("precision", "fp64")]
    pb.quad_rule = QUAD[spec.get("quad_rule", "gl")]
    pb.hessian_reuse = int(spec.get("hessian_reuse", 0))
    pb.reuse_theta = float(spec.get("reuse_theta", 0.0))
    pb.adapt = int(spec.get("adapt", 0))
    pb.min_degree = spec.get("min_degree", 1)
    pb.delta_lo = spec.get("delta_lo", 0.0)
    pb.delta_hi = spec.get("delta_hi", 0.0)
    stages = spec.get("retard", ())  # [(max degree, residual tolerance), ...]
    pb.n_retard = len(stages)
    if stages:
        dg = (C.c_int * len(stages))(*[int(d) for d, _ in stages])
        ep = (C.c_double * len(stages))(*[float(e) for _, e in stages])
        keep.extend([dg, ep])
        pb.retard_degree = C.cast(dg, C.POINTER(C.c_int))
        pb.retard_eps = C.cast(ep, C.POINTER(C.c_double))
    pb.nx = spec["nx"]
    pb.ny = spec.get("ny", 1)
    pb.x0, pb.x1 = spec["x0"], spec["x1"]
    pb.y0, pb.y1 = spec.get("y0", 0.0), spec.get("y1", 1.0)
    for k, b in enumerate(spec["bc"][:4]):
        pb.bc[k] = BC[b]
    return pb


class Context:
    """A libipm context on one device, ordered on one HIP stream."""

    def __init__(self, device=0, stream=None, hbm_budget=0, max_problems=0):
        self.lib = load()
        cfg = Config()
        cfg.device = device
        cfg.hip_stream = stream
        cfg.hbm_budget_bytes = hbm_budget
        cfg.max_problems = max_problems
        h = C.c_void_p()
        st = self.lib.ipm_create(C.byref(cfg), C.byref(h))
        if st != 0:
            raise IpmError(st, self.lib.ipm_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != 0:
            raise IpmError(st, self.lib.ipm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.ipm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _problem(spec, keep, ic_nodal=None, ic_moments=None, ic_dual=None, dirichlet=None,
                 cell_degree=None):
        pb = problem_struct(spec, keep)

        def arr(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            return _dptr(a)

        pb.ic_nodal = arr(ic_nodal)
        pb.ic_moments = arr(ic_moments)
        pb.ic_dual = arr(ic_dual)
        pb.dirichlet = arr(dirichlet)
        if cell_degree is not None:
            cd = np.ascontiguousarray(cell_degree, dtype=np.int8)
            keep.append(cd)
            pb.cell_degree = cd.ctypes.data_as(C.POINTER(C.c_int8))
        keep.append(pb)
        return pb

    def set_problem(self, spec, ic_nodal=None, ic_moments=None, ic_dual=None, dirichlet=None,
                    cell_degree=None):
        keep = []
        pb = self._problem(spec, keep, ic_nodal, ic_moments, ic_dual, dirichlet, cell_degree)
        pid = C.c_int(-1)
        self._check(self.lib.ipm_set_problem(self.h, C.byref(pb), C.byref(pid)))
        return pid.value

    def serve(self, requests, steps_per_round=8, max_active=64, moments=True):
        """Run a request stream through ipm_serve.  requests: list of dicts with
        'spec', 'arrival' (s) and the set_problem keyword arrays ('ic_nodal',
        ...).  Returns one dict per request: admitted, finished, latency,
        steps, status and (if moments) the final moments."""
        keep = []
        reqs = (Request * len(requests))()
        outs = []
        for k, rq in enumerate(requests):
            kw = {key: rq.get(key) for key in ("ic_nodal", "ic_moments", "ic_dual", "dirichlet",
                                               "cell_degree")}
            pb = self._problem(rq["spec"], keep, **kw)
            reqs[k].problem = C.cast(C.pointer(pb), C.c_void_p)
            reqs[k].arrival_s = float(rq["arrival"])
            out = None
            if moments:
                m = {"burgers1d": 1, "euler1d": 3, "euler2d": 4}[rq["spec"]["equation"]]
                cells = rq["spec"]["nx"] * (rq["spec"].get("ny", 1) if m == 4 else 1)
                N = self.lib.ipm_basis_size(rq["spec"]["p"], rq["spec"]["degree"])
                out = np.zeros((cells, m, N))
                reqs[k].moments_out = _dptr(out)
                reqs[k].moments_len = out.size
            outs.append(out)
        self._check(self.lib.ipm_serve(self.h, len(requests), reqs, int(steps_per_round),
                                       int(max_active)))
        res = []
        for k, rq in enumerate(requests):
            r = reqs[k]
            res.append({"admitted": r.admitted_s, "finished": r.finished_s,
                        "latency": r.finished_s - r.arrival_s, "steps": r.steps,
                        "status": r.status, "moments": outs[k]})
        return res

    def footprint(self, spec):
        return self.lib.ipm_problem_footprint(C.byref(problem_struct(spec, [])))

    def step(self, ids, max_steps, wait=False):
        ids = [ids] if isinstance(ids, int) else list(ids)
        arr = (C.c_int * len(ids))(*ids)
        infos = (StepInfo * len(ids))() if wait else None
        self._check(self.lib.ipm_step(self.h, len(ids), arr, int(max_steps), infos))
        return [i.as_dict() for i in infos] if wait else None

    def step_static(self, ids, max_steps, wait=False):
        """ipm_step_static: the batched step without device allocations."""
        ids = [ids] if isinstance(ids, int) else list(ids)
        arr = (C.c_int * len(ids))(*ids)
        infos = (StepInfo * len(ids))() if wait else None
        self._check(self.lib.ipm_step_static(self.h, len(ids), arr, int(max_steps), infos))
        return [i.as_dict() for i in infos] if wait else None

    def query(self, pid):
        info = StepInfo()
        self._check(self.lib.ipm_query(self.h, pid, C.byref(info)))
        return info.as_dict()

    def sizes(self, pid):
        m, N, Q, cells = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        self._check(self.lib.ipm_problem_sizes(self.h, pid, C.byref(m), C.byref(N), C.byref(Q),
                                               C.byref(cells)))
        return m.value, N.value, Q.value, cells.value

    def moments(self, pid, out=None):
        """Moments [cells][m][N] as NumPy (host) or into a torch CUDA tensor."""
        m, N, _, cells = self.sizes(pid)
        if out is None:
            out = np.zeros((cells, m, N))
            self._check(self.lib.ipm_moments(self.h, pid, out.ctypes.data, out.size, 0))
            return out
        self._check(self.lib.ipm_moments(self.h, pid, C.c_void_p(out.data_ptr()), out.numel(), 1))
        return out

    def dual(self, pid):
        m, N, _, cells = self.sizes(pid)
        out = np.zeros((cells, m, N))
        self._check(self.lib.ipm_dual(self.h, pid, out.ctypes.data, out.size, 0))
        return out

    def degrees(self, pid):
        """Current total degree (refinement level) of every cell."""
        _, _, _, cells = self.sizes(pid)
        out = np.zeros(cells, dtype=np.int8)
        self._check(self.lib.ipm_cell_degrees(self.h, pid, out.ctypes.data_as(C.POINTER(C.c_int8)),
                                              cells))
        return out

    def release(self, pid):
        self._check(self.lib.ipm_release(self.h, pid))

    def autotune(self, ids, steps_per_candidate=4):
        """Pick the wavefronts per Newton block of every small-cell kernel shape
        by timing real steps of the problems `ids` (see ipm_autotune)."""
        ids = list(ids)
        arr = (C.c_int * len(ids))(*ids)
        n = C.c_int()
        self._check(self.lib.ipm_autotune(self.h, len(ids), arr, int(steps_per_candidate), C.byref(n)))
        return n.value

    def launch_times(self):
        """Per Newton kernel shape: launches and device ms of the last timing window."""
        n = C.c_int()
        buf = (LaunchTime * 64)()
        self._check(self.lib.ipm_launch_times(self.h, buf, 64, C.byref(n)))
        return [buf[k].as_dict() for k in range(min(n.value, 64))]

    def class_stats(self, pid):
        """Cumulative Newton counters per size class of a problem."""
        n = C.c_int()
        buf = (ClassStat * 16)()
        self._check(self.lib.ipm_class_stats(self.h, pid, buf, 16, C.byref(n)))
        return [buf[k].as_dict() for k in range(min(n.value, 16))]

    def timing(self, enable):
        d, u, n = C.c_double(), C.c_double(), C.c_longlong()
        self._check(self.lib.ipm_kernel_timing(self.h, int(enable), C.byref(d), C.byref(u), C.byref(n)))
        return {"dual_ms": d.value, "update_ms": u.value, "launches": n.value}
