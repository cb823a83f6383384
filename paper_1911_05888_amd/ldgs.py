"""ctypes binding of libldgs.so (the C ABI declared in include/ldgs.h).

Argument marshalling only: every computation runs in the library.  Device
vectors are torch tensors (float64, on the GPU); the library works on the
stream that was current when the context was created.  Importing this module
fails loudly if the compiled library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libldgs.so not found at {LIB_PATH}: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")
# PyTorch first: the library then binds to the HIP runtime PyTorch loads, so
# that both share one runtime (streams, allocations) whatever the caller
# imports first
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

# status codes
OK, E_ARG, E_UNSUPPORTED, E_NOMEM, E_HIP, E_SINGULAR_BLOCK, E_COLORING, E_NOT_CONVERGED, E_NONFINITE = range(9)
STANDARD, VISCOUS_STRESS = 0, 1
PERIODIC, DIRICHLET, STRESS = 0, 1, 2
COLOR_AUTO, COLOR_RED_BLACK, COLOR_PARITY, COLOR_MOD3 = 0, 1, 2, 3
V_FP64, V_FP32, V_FP32_BF16BLK = 0, 1, 2
STATIONARY, IR, FGMRES, GMRES = 0, 1, 2, 3
FIELD_CONST, FIELD_SINSIN, FIELD_LOGNORMAL_RFF, FIELD_PHASE_CONST, FIELD_CALLBACK = range(5)
LEVELSET_NONE, LEVELSET_BOX, LEVELSET_CIRCLE, LEVELSET_DISK = 0, 1, 2, 3
NET_HIDDEN = 16          # hidden width of the learned correction network
TRAIN_WORKSPACE_BYTES = 4 << 20   # workspace of ldgs_learned_train_noalloc (LDGS_TRAIN_WORKSPACE_BYTES)

EVAL_FN = C.CFUNCTYPE(None, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int),
                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Field(C.Structure):
    _fields_ = [("kind", C.c_int), ("params", C.POINTER(C.c_double)), ("nparams", C.c_int64),
                ("fn", EVAL_FN), ("user", C.c_void_p)]


class ProblemStruct(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("degree", C.c_int), ("form", C.c_int),
                ("bc", C.c_int * 3), ("mu", Field), ("rho", Field), ("delta", C.c_double),
                ("levelset_kind", C.c_int), ("levelset_params", C.c_double * 2),
                ("tau", C.c_double), ("tau0", C.c_double), ("tau_u_bdry_C", C.c_double),
                ("tau_u_inter_C", C.c_double), ("nu1", C.c_int), ("nu2", C.c_int),
                ("coarsest_n", C.c_int), ("coloring", C.c_int), ("vprec", C.c_int),
                ("build_precisions", C.c_int), ("diag_scaling", C.c_int), ("host_only", C.c_int),
                ("hip_stream", C.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_user", C.c_void_p), ("levelset_centre", C.c_double * 3),
                ("tau_u_intra_C", C.c_double), ("q_cut", C.c_int)]


class RhsData(C.Structure):
    _fields_ = [("f", EVAL_FN), ("f_div", EVAL_FN), ("g_dirichlet", EVAL_FN), ("g_jump", EVAL_FN),
                ("h_jump", EVAL_FN), ("h_stress", EVAL_FN), ("user", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("fallback_events", C.c_int), ("relres", C.c_double),
                ("rho_measured", C.c_double), ("t_solve_s", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int), ("history_len", C.c_int)]


class NetStruct(C.Structure):
    _fields_ = [("dim", C.c_int), ("degree", C.c_int), ("hidden", C.c_int), ("params", C.POINTER(C.c_float)),
                ("nparams", C.c_int64), ("c_vel", C.c_double), ("c_pre", C.c_double)]


class TrainArgs(C.Structure):
    _fields_ = [("hip_stream", C.c_void_p), ("dim", C.c_int), ("degree", C.c_int), ("hidden", C.c_int),
                ("crop", C.c_int), ("ncrops", C.c_int), ("feat", C.c_void_p), ("targ", C.c_void_p),
                ("c_vel", C.c_double), ("c_pre", C.c_double), ("batch", C.c_int), ("steps", C.c_int),
                ("order", C.POINTER(C.c_int)), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "ldgs_setup": ([C.POINTER(ProblemStruct), C.POINTER(C.c_void_p)]),
    "ldgs_num_dofs": ([_P, C.POINTER(C.c_int64)]),
    "ldgs_assemble_rhs": ([_P, C.POINTER(RhsData), _P]),
    "ldgs_apply": ([_P, _P, _P]),
    "ldgs_residual": ([_P, _P, _P, _P, _D]),
    "ldgs_vcycle": ([_P, _P, _P]),
    "ldgs_solve": ([_P, _P, _P, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(Info)]),
    "ldgs_set_vprec": ([_P, C.c_int]),
    "ldgs_graph_count": ([_P, C.POINTER(C.c_int)]),
    "ldgs_gmres_rho": ([_P, _P, C.c_double, C.c_int, _D, C.POINTER(C.c_int), _D, C.c_int]),
    "ldgs_set_learned": ([_P, C.POINTER(NetStruct)]),
    "ldgs_learned_correction": ([_P, _P, _P]),
    "ldgs_learned_collect": ([_P, _P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), _P, _P, _D]),
    "ldgs_learned_train": ([C.POINTER(TrainArgs), C.POINTER(C.c_float), _D, C.POINTER(C.c_float)]),
    "ldgs_learned_train_noalloc": ([C.POINTER(TrainArgs), C.POINTER(C.c_float), _D, C.POINTER(C.c_float)]),
    "ldgs_project_kernel": ([_P, _P]),
    "ldgs_level_info": ([_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ldgs_level_elements": ([_P, C.c_int, C.POINTER(C.c_int64)]),
    "ldgs_level_blocks": ([_P, C.c_int, C.POINTER(C.c_int64)]),
    "ldgs_level_shared_inverse": ([_P, C.c_int, C.POINTER(C.c_int)]),
    "ldgs_level_smooth_colour": ([_P, C.c_int, C.c_int, _P, _P]),
    "ldgs_level_residual_restrict": ([_P, C.c_int, _P, _P, _P]),
    "ldgs_level_prolong_add": ([_P, C.c_int, _P, _P]),
    "ldgs_bottom_solve": ([_P, _P, _P]),
    "ldgs_level_apply": ([_P, C.c_int, _P, _P]),
    "ldgs_level_block_inverse": ([_P, C.c_int, C.c_int64, _D]),
    "ldgs_host_level_apply": ([_P, C.c_int, _D, _D]),
    "ldgs_bottom_info": ([_P, C.POINTER(C.c_int64), _D, _D]),
    "ldgs_level_smooth_colour_f32": ([_P, C.c_int, C.c_int, C.c_int, _P, _P]),
    "ldgs_profile": ([_P, C.c_int]),
    "ldgs_profile_read": ([_P, _D, C.POINTER(C.c_int64)]),
    "ldgs_destroy": ([_P]),
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.ldgs_status_str.argtypes = [C.c_int]
_lib.ldgs_status_str.restype = C.c_char_p
_lib.ldgs_last_error.argtypes = [_P]
_lib.ldgs_last_error.restype = C.c_char_p

EXPORTED = sorted(list(_SIGS) + ["ldgs_status_str", "ldgs_last_error"])


class LdgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.ldgs_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def _dptr(t):
    """Device pointer of a torch tensor (or host pointer of a numpy array)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def _np_eval(fn, ncomp, dim):
    """Wraps fn(x (n,d), phase (n,), normal or None) -> (n, ncomp) as a C callback."""
    def cb(n, x, phase, normal, out, user):
        xa = np.ctypeslib.as_array(x, shape=(n, dim))
        ph = np.ctypeslib.as_array(phase, shape=(n,)) if phase else None
        nr = np.ctypeslib.as_array(normal, shape=(n, dim)) if normal else None
        val = np.asarray(fn(xa, ph, nr), dtype=np.float64).reshape(n, ncomp)
        np.ctypeslib.as_array(out, shape=(n, ncomp))[:] = val
    return EVAL_FN(cb)


def _field(obj, dim, keep):
    """ldgs_field from a coefficient object with ``kind`` and ``params()``."""
    kind = {"const": FIELD_CONST, "sinsin": FIELD_SINSIN, "lognormal_rff": FIELD_LOGNORMAL_RFF,
            "phase": FIELD_PHASE_CONST, "circle": FIELD_PHASE_CONST}.get(getattr(obj, "kind", None), FIELD_CALLBACK)
    f = Field()
    f.kind = kind
    if kind == FIELD_CALLBACK:
        cb = _np_eval(lambda x, ph, nr: obj.value(x, ph), 1, dim)
        keep.append(cb)
        f.fn = cb
    else:
        pr = np.ascontiguousarray(obj.params(), dtype=np.float64)
        if kind == FIELD_PHASE_CONST:
            pr = pr[:2].copy()
        keep.append(pr)
        f.params = pr.ctypes.data_as(C.POINTER(C.c_double))
        f.nparams = pr.size
    return f


def torch_allocator(device=None, stream=None):
    """(dev_alloc, dev_free) callbacks drawing the context's device storage
    from PyTorch's caching allocator, so that PyTorch stays the owner of the
    memory (it shows in torch.cuda.memory_allocated())."""
    import torch

    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:          # out of memory: the library reports LDGS_E_NOMEM
            return None

    def free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:          # interpreter shutdown: the process frees the memory
            pass
    return ALLOC_FN(alloc), FREE_FN(free)


def problem_struct(prob, vprec=V_FP64, build_precisions=0, host_only=False, stream=None, coloring=None,
                   allocator=None):
    """ldgs_problem from a problem description object (attributes dim, n, p,
    gamma, bc, mu, rho, delta, phases, tau, tau0, tau_u_bdry_C, tau_u_inter_C,
    nu1, nu2, coarsest_n, coloring, diag_scaling).  Returns (struct, keepalive)."""
    keep = []
    s = ProblemStruct()
    s.dim, s.n, s.degree, s.form = prob.dim, prob.n, prob.p, prob.gamma
    for j, b in enumerate(prob.bc):
        s.bc[j] = {"periodic": PERIODIC, "dirichlet": DIRICHLET, "stress": STRESS}[b]
    s.mu = _field(prob.mu, prob.dim, keep)
    if getattr(prob, "rho", None) is not None:
        s.rho = _field(prob.rho, prob.dim, keep)
    s.delta = prob.delta if getattr(prob, "delta", None) else 0.0
    ph = getattr(prob, "phases", None)
    if ph is not None and getattr(ph, "kind", None) == "circle":
        s.levelset_kind = LEVELSET_DISK if getattr(ph, "void_outside", False) else LEVELSET_CIRCLE
        s.levelset_params[0] = ph.radius
        s.levelset_centre[0], s.levelset_centre[1] = ph.centre
        s.tau_u_intra_C = getattr(prob, "tau_u_intra_C", 0.0)
        s.q_cut = getattr(prob, "q_cut", 8)
    elif ph is not None:
        s.levelset_kind = LEVELSET_BOX
        s.levelset_params[0] = ph.lo
        s.levelset_params[1] = ph.hi
    s.tau, s.tau0 = prob.tau, prob.tau0
    s.tau_u_bdry_C, s.tau_u_inter_C = prob.tau_u_bdry_C, prob.tau_u_inter_C
    s.nu1, s.nu2, s.coarsest_n = prob.nu1, prob.nu2, prob.coarsest_n
    col = coloring if coloring is not None else prob.coloring
    s.coloring = {"auto": COLOR_AUTO, "rb": COLOR_RED_BLACK, "parity": COLOR_PARITY,
                  "mod3": COLOR_MOD3, "greedy": COLOR_AUTO}.get(col, col)
    s.vprec = vprec
    s.build_precisions = build_precisions
    s.diag_scaling = int(bool(getattr(prob, "diag_scaling", False)))
    s.host_only = int(bool(host_only))
    s.hip_stream = stream
    if allocator is not None:
        s.dev_alloc, s.dev_free = allocator
        keep.extend(allocator)
    return s, keep


def rhs_callbacks(src, dim):
    """ldgs_rhs_data from a data object providing forcing(x, chi) (d comps),
    forcing_div(x, chi), and, if it is an exact solution, velocity(x, chi)
    and stress(x, chi) (Dirichlet data and interface jumps)."""
    keep = []
    r = RhsData()

    def mk(fn, ncomp):
        cb = _np_eval(fn, ncomp, dim)
        keep.append(cb)
        return cb

    r.f = mk(lambda x, ph, nr: src.forcing(x, ph), dim)
    r.f_div = mk(lambda x, ph, nr: src.forcing_div(x, ph), 1)
    if hasattr(src, "interface_jumps"):
        r.g_dirichlet = mk(lambda x, ph, nr: src.velocity(x, ph), dim)
        r.g_jump = mk(lambda x, ph, nr: src.interface_jumps(x, nr)[0], dim)
        r.h_jump = mk(lambda x, ph, nr: src.interface_jumps(x, nr)[1], dim)
    elif hasattr(src, "velocity"):
        r.g_dirichlet = mk(lambda x, ph, nr: src.velocity(x, ph), dim)

        def gj(x, ph, nr):
            return src.velocity(x, np.ones_like(ph)) - src.velocity(x, 2 * np.ones_like(ph))

        def hj(x, ph, nr):
            sd = src.stress(x, np.ones_like(ph)) - src.stress(x, 2 * np.ones_like(ph))
            return np.einsum("nij,nj->ni", sd, nr)
        r.g_jump = mk(gj, dim)
        r.h_jump = mk(hj, dim)
        # stress walls: h = sigma n, n the outward normal the library passes
        r.h_stress = mk(lambda x, ph, nr: np.einsum("nij,nj->ni", src.stress(x, ph), nr), dim)
    return r, keep


class Context:
    """One ldgs context (levels, smoother data, bottom solver) on the GPU, or on
    the host only when ``host_only`` is set (setup validation)."""

    def __init__(self, prob, vprec=V_FP64, build_precisions=0, host_only=False, coloring=None,
                 torch_memory=True):
        """The context works on the current torch stream (on the default
        stream the library uses a stream of its own, joined to the default
        one at every call).  torch_memory: draw every device allocation of
        the context from PyTorch's caching allocator."""
        stream = None
        allocator = None
        self.host_only = host_only
        if not host_only:
            import torch
            cur = torch.cuda.current_stream()
            stream = C.c_void_p(cur.cuda_stream) if cur.cuda_stream else None
            if torch_memory:
                allocator = torch_allocator(torch.cuda.current_device(), cur)
        self.prob = prob
        self._s, self._keep = problem_struct(prob, vprec, build_precisions, host_only, stream, coloring,
                                             allocator)
        h = C.c_void_p()
        st = _lib.ldgs_setup(C.byref(self._s), C.byref(h))
        if st != OK:
            raise LdgsError(st, _lib.ldgs_last_error(None).decode())
        self._h = h
        n = C.c_int64()
        self._check(_lib.ldgs_num_dofs(self._h, C.byref(n)))
        self.ndof = n.value
        nl = C.c_int()
        self._check(_lib.ldgs_level_info(self._h, 0, None, C.byref(nl), None))
        self.n_levels = nl.value

    def _check(self, st):
        if st != OK:
            raise LdgsError(st, _lib.ldgs_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None):
            _lib.ldgs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- main entry points ------------------------------------------------
    def zeros(self, n=None):
        import torch
        return torch.zeros(self.ndof if n is None else n, dtype=torch.float64, device="cuda")

    def assemble_rhs(self, src, out=None):
        r, keep = rhs_callbacks(src, self.prob.dim)
        if out is None:
            out = np.zeros(self.ndof) if self.host_only else self.zeros()
        self._check(_lib.ldgs_assemble_rhs(self._h, C.byref(r), _dptr(out)))
        return out

    def apply(self, x, y=None):
        y = self.zeros() if y is None else y
        self._check(_lib.ldgs_apply(self._h, _dptr(x), _dptr(y)))
        return y

    def residual(self, b, x, r=None):
        nrm = C.c_double()
        self._check(_lib.ldgs_residual(self._h, _dptr(b), _dptr(x), _dptr(r), C.byref(nrm)))
        return nrm.value

    def vcycle(self, b, x):
        self._check(_lib.ldgs_vcycle(self._h, _dptr(b), _dptr(x)))
        return x

    def set_vprec(self, vprec):
        self._check(_lib.ldgs_set_vprec(self._h, vprec))

    def gmres_rho(self, x0, reduction=1e-8, maxit=200):
        """rho of eq. (rho) from the initial guess x0 (device FP64, b = 0).
        Returns (rho, iterations, history of ||V A x_k|| / ||V A x_0||,
        converged)."""
        rho, its = C.c_double(), C.c_int()
        hist = np.zeros(maxit + 1)
        st = _lib.ldgs_gmres_rho(self._h, _dptr(x0), reduction, maxit, C.byref(rho), C.byref(its),
                                 hist.ctypes.data_as(_D), hist.size)
        if st not in (OK, E_NOT_CONVERGED):
            self._check(st)
        return rho.value, its.value, hist[:its.value + 1].copy(), st == OK

    def graph_count(self):
        """V-cycles captured into HIP graphs so far (0: direct launches)."""
        v = C.c_int()
        self._check(_lib.ldgs_graph_count(self._h, C.byref(v)))
        return v.value

    def project_kernel(self, v):
        self._check(_lib.ldgs_project_kernel(self._h, _dptr(v)))
        return v

    def solve(self, b, x, tol=1e-10, maxit=100, outer=STATIONARY, fgmres_m=30, use_learned=False,
              history_cap=512, raise_on_failure=False):
        """Returns (status, info dict).  b is projected onto range(A) in place."""
        hist = (C.c_double * history_cap)()
        info = Info()
        info.history = C.cast(hist, C.POINTER(C.c_double))
        info.history_cap = history_cap
        st = _lib.ldgs_solve(self._h, _dptr(b), _dptr(x), tol, maxit, outer, fgmres_m,
                             int(bool(use_learned)), C.byref(info))
        if st != OK and (raise_on_failure or st not in (E_NOT_CONVERGED,)):
            self._check(st)
        return st, dict(iters=info.iters, relres=info.relres, rho=info.rho_measured,
                        t_solve_s=info.t_solve_s, fallback_events=info.fallback_events,
                        history=np.array(hist[:info.history_len]))

    # ---- learned correction -------------------------------------------------
    def set_learned(self, params, c_vel, c_pre, hidden=NET_HIDDEN):
        """params: flat FP32 array in the layout of ldgs_net (or None to remove)."""
        if params is None:
            self._check(_lib.ldgs_set_learned(self._h, None))
            return
        flat = np.ascontiguousarray(params, dtype=np.float32)
        net = NetStruct(self.prob.dim, self.prob.p, hidden, flat.ctypes.data_as(C.POINTER(C.c_float)),
                        flat.size, c_vel, c_pre)
        self._check(_lib.ldgs_set_learned(self._h, C.byref(net)))

    def learned_correction(self, r, dx=None):
        dx = self.zeros() if dx is None else dx
        self._check(_lib.ldgs_learned_correction(self._h, _dptr(r), _dptr(dx)))
        return dx

    def learned_collect(self, xstar, ncycles, crop, origins):
        """origins: int array (ncycles, ncrops, d).  Returns (feat, targ, stats):
        feat/targ device int16 tensors holding bfloat16 bits, stats (ncycles, 4)."""
        import torch
        org = np.ascontiguousarray(origins, dtype=np.int32)
        ncrops = org.shape[1]
        d = self.prob.dim
        nb = (d + 1) * (self.prob.p + 1) ** d
        chp = (nb + 1 + 7) // 8 * 8
        feat = torch.empty(ncycles * ncrops * (crop + 2) ** d * chp, dtype=torch.int16, device="cuda")
        targ = torch.empty(ncycles * ncrops * crop ** d * nb, dtype=torch.int16, device="cuda")
        stats = np.zeros((ncycles, 4))
        self._check(_lib.ldgs_learned_collect(self._h, _dptr(xstar), ncycles, crop, ncrops,
                                              org.ctypes.data_as(C.POINTER(C.c_int)), _dptr(feat), _dptr(targ),
                                              stats.ctypes.data_as(_D)))
        return feat, targ, stats

    # ---- stages -------------------------------------------------------------
    def level_info(self, level):
        n, nl, nc = C.c_int(), C.c_int(), C.c_int()
        self._check(_lib.ldgs_level_info(self._h, level, C.byref(n), C.byref(nl), C.byref(nc)))
        return n.value, nl.value, nc.value

    def level_elements(self, level):
        ne = C.c_int64()
        self._check(_lib.ldgs_level_elements(self._h, level, C.byref(ne)))
        return ne.value

    def level_blocks(self, level):
        nbk = C.c_int64()
        self._check(_lib.ldgs_level_blocks(self._h, level, C.byref(nbk)))
        return nbk.value

    def level_shared_inverse(self, level):
        v = C.c_int()
        self._check(_lib.ldgs_level_shared_inverse(self._h, level, C.byref(v)))
        return bool(v.value)

    def level_smooth_colour(self, level, colour, b, x):
        self._check(_lib.ldgs_level_smooth_colour(self._h, level, colour, _dptr(b), _dptr(x)))

    def level_smooth_colour_f32(self, level, colour, vprec, b, x):
        self._check(_lib.ldgs_level_smooth_colour_f32(self._h, level, colour, vprec, _dptr(b), _dptr(x)))

    def profile(self, stride=1):
        """Time every `stride`-th finest sweep, one event pair around all its
        colour passes (True: every sweep; 0 or False: off)."""
        self._check(_lib.ldgs_profile(self._h, int(stride)))

    def profile_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(_lib.ldgs_profile_read(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def level_residual_restrict(self, level, b, x, rc):
        self._check(_lib.ldgs_level_residual_restrict(self._h, level, _dptr(b), _dptr(x), _dptr(rc)))

    def level_prolong_add(self, level, xc, x):
        self._check(_lib.ldgs_level_prolong_add(self._h, level, _dptr(xc), _dptr(x)))

    def bottom_solve(self, b, x):
        self._check(_lib.ldgs_bottom_solve(self._h, _dptr(b), _dptr(x)))

    def level_apply(self, level, x, y):
        self._check(_lib.ldgs_level_apply(self._h, level, _dptr(x), _dptr(y)))

    def level_block_inverse(self, level, element):
        nb = (self.prob.dim + 1) * (self.prob.p + 1) ** self.prob.dim
        out = np.zeros((nb, nb))
        self._check(_lib.ldgs_level_block_inverse(self._h, level, element,
                                                  out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def host_level_apply(self, level, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        self._check(_lib.ldgs_host_level_apply(self._h, level, x.ctypes.data_as(C.POINTER(C.c_double)),
                                               y.ctypes.data_as(C.POINTER(C.c_double))))
        return y

    def bottom_info(self):
        nc = C.c_int64()
        self._check(_lib.ldgs_bottom_info(self._h, C.byref(nc), None, None))
        pinv = np.zeros((nc.value, nc.value))
        eig = np.zeros(nc.value)
        self._check(_lib.ldgs_bottom_info(self._h, None, pinv.ctypes.data_as(C.POINTER(C.c_double)),
                                          eig.ctypes.data_as(C.POINTER(C.c_double))))
        return pinv, eig


def net_nparams(dim, degree, hidden=NET_HIDDEN):
    nb = (dim + 1) * (degree + 1) ** dim
    return hidden * 3 ** dim * (nb + 1) + 2 * hidden + hidden * hidden + nb * hidden + nb


def learned_train(dim, degree, crop, ncrops, feat, targ, c_vel, c_pre, params, order, lr=1e-3,
                  beta1=0.9, beta2=0.999, eps=1e-8, want_grad0=False, hidden=NET_HIDDEN, noalloc=False):
    """Runs len(order) Adam steps (order: int array (steps, batch) of crop
    indices) on device crops; returns (params, losses, grad0 or None).
    noalloc: use the entry point that allocates no device memory (fixed
    per-GPU workspace of TRAIN_WORKSPACE_BYTES)."""
    import torch
    p = np.array(params, dtype=np.float32, copy=True)
    org = np.ascontiguousarray(order, dtype=np.int32)
    if org.ndim != 2:
        raise ValueError("order must be (steps, batch)")
    steps, batch = org.shape
    a = TrainArgs(C.c_void_p(torch.cuda.current_stream().cuda_stream), dim, degree, hidden, crop, ncrops,
                  _dptr(feat), _dptr(targ), c_vel, c_pre, batch, steps,
                  org.ctypes.data_as(C.POINTER(C.c_int)), lr, beta1, beta2, eps)
    losses = np.zeros(max(steps, 1))
    g0 = np.zeros_like(p) if want_grad0 else None
    fn = _lib.ldgs_learned_train_noalloc if noalloc else _lib.ldgs_learned_train
    st = fn(C.byref(a), p.ctypes.data_as(C.POINTER(C.c_float)), losses.ctypes.data_as(_D),
            g0.ctypes.data_as(C.POINTER(C.c_float)) if want_grad0 else None)
    if st != OK:
        raise LdgsError(st, _lib.ldgs_last_error(None).decode())
    return p, losses[:steps], g0


def init_net_params(dim, degree, seed, hidden=NET_HIDDEN, out_scale=0.1):
    """He-normal initial weights in the flat layout of ldgs_net (zero biases;
    the output layer scaled by out_scale)."""
    nb = (dim + 1) * (degree + 1) ** dim
    K = 3 ** dim * (nb + 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.standard_normal(hidden * K) * np.sqrt(2.0 / K), np.zeros(hidden),
             rng.standard_normal(hidden * hidden) * np.sqrt(2.0 / hidden), np.zeros(hidden),
             out_scale * rng.standard_normal(nb * hidden) * np.sqrt(1.0 / hidden), np.zeros(nb)]
    return np.concatenate(parts).astype(np.float32)
