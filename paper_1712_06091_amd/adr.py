"""Thin Python binding of libadr (the C ABI in include/adr.h).

Argument marshalling only: every step of the solve runs in the HIP library.  PyTorch
provides device memory and the stream.  Arrays follow the library layout: C-ordered
(nz, ny, nx) / (ny, nx) tensors with x fastest; complex data as torch.complex128.
Source indices are given in the same (NumPy) axis order and reversed for the ABI, whose
axis 0 is x.

There is no CPU fallback: if libadr.so is missing or fails to load, every call raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadr.so")

ADR_OK, ADR_EINVAL, ADR_ENOMEM, ADR_EHIP, ADR_ENOCONV, ADR_ENUMERIC, ADR_ENOTSUP = range(7)
ADR_PREC_FP64, ADR_PREC_MIXED = 0, 1
ADR_RELAX_JACOBI, ADR_RELAX_GMRES = 0, 1
ADR_CYCLE_V, ADR_CYCLE_K = 0, 1
ADR_ADV_UPWIND, ADR_ADV_CENTRAL = 0, 1
ADR_REACTION_NUMERICAL, ADR_REACTION_EIKONAL = 0, 1
ADR_NOALLOC_MAX_REC = 1 << 26
TIMER_KINDS = {"fine_jacobi": 0, "fine_residual": 1, "coarse_apply": 2, "coarse_orth": 3, "transfer": 4,
               "outer_matvec": 5, "outer_orth": 6, "coarse_tail": 7, "fine_gmres": 8}


class AdrProblem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("kappa2", ctypes.c_void_p),
        ("tau", ctypes.c_void_p),
        ("gamma", ctypes.c_void_p),
        ("src", ctypes.c_int * 3),
    ]


class AdrOptions(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("coarsest_max", ctypes.c_int),
        ("nu", ctypes.c_int * 8),
        ("relax", ctypes.c_int * 8),
        ("jacobi_weight", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("restart", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("cycle", ctypes.c_int),
        ("kcycle_threshold", ctypes.c_double),
        ("coarse_split", ctypes.c_int),
        ("tail_max_nodes", ctypes.c_int),
        ("full_cycles", ctypes.c_int),
        ("shift_alpha", ctypes.c_double),
        ("advection", ctypes.c_int),
        ("outer_beta", ctypes.c_double),
        ("rescaled", ctypes.c_int),
        ("pipeline_max_nodes", ctypes.c_int),
        ("reaction", ctypes.c_int),
        ("kcycle_levels", ctypes.c_int),
        ("fine_tiles", ctypes.c_int),
        ("batch_merge", ctypes.c_int),
    ]


class AdrStats(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("relres", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class AdrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load_library(path=LIB_PATH):
    """Load libadr.so once; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libadr.so not found at {path}: run __graft_entry__.build() "
                           "(python -m paper_1712_06091_amd.build)")
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "adr_default_options": (None, [ctypes.POINTER(AdrOptions)]),
        "adr_setup": (I, [ctypes.POINTER(AdrProblem), ctypes.POINTER(AdrOptions), P, ctypes.POINTER(P)]),
        "adr_destroy": (None, [P]),
        "adr_apply": (I, [P, D, P, P]),
        "adr_vcycle": (I, [P, P, P]),
        "adr_solve": (I, [P, P, P, D, I, I, ctypes.POINTER(AdrStats)]),
        "adr_two_stage_options": (None, [ctypes.POINTER(AdrOptions), ctypes.POINTER(AdrOptions)]),
        "adr_solve_two_stage": (I, [P, P, P, P, D, I, D, I, ctypes.POINTER(AdrStats), ctypes.POINTER(AdrStats)]),
        "adr_wavefield": (I, [P, P, P]),
        "adr_get_coefficients": (I, [P, P, P, P]),
        "adr_level_info": (I, [P, I, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "adr_level_split": (I, [P, I, ctypes.POINTER(ctypes.c_int)]),
        "adr_num_levels": (I, [P]),
        "adr_tuning_table_write": (I, [ctypes.c_char_p]),
        "adr_tuning_table_read": (I, [ctypes.c_char_p]),
        "adr_get_level_stencil": (I, [P, I, P, ctypes.POINTER(ctypes.c_int)]),
        "adr_solve_adjoint": (I, [P, P, P, D, I, I, ctypes.POINTER(AdrStats)]),
        "adr_apply_adjoint": (I, [P, P, P]),
        "adr_grad_kappa2": (I, [P, P, P, P]),
        "adr_receiver_residual": (I, [P, P, P, P, I, P, ctypes.POINTER(ctypes.c_double)]),
        "adr_receiver_residual_noalloc": (I, [P, P, P, I, P, ctypes.POINTER(ctypes.c_double), P]),
        "adr_adjoint_source": (I, [P, P, P, I, P]),
        "adr_eikonal": (I, [I, ctypes.POINTER(ctypes.c_int), D, P, ctypes.POINTER(ctypes.c_int), P, P, I,
                            ctypes.POINTER(ctypes.c_int), P]),
        "adr_setup_batch": (I, [I, ctypes.POINTER(AdrProblem), ctypes.POINTER(AdrOptions), I, ctypes.POINTER(P)]),
        "adr_solve_batch": (I, [P, ctypes.POINTER(P), ctypes.POINTER(P), D, I, ctypes.POINTER(AdrStats)]),
        "adr_batch_size": (I, [P]),
        "adr_batch_groups": (I, [P]),
        "adr_batch_context": (P, [P, I]),
        "adr_destroy_batch": (None, [P]),
        "adr_timer_start": (I, [P, I, I]),
        "adr_timer_stop": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_double)]),
        "adr_strerror": (ctypes.c_char_p, [I]),
        "adr_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_options(**kw):
    lib = load_library()
    o = AdrOptions()
    lib.adr_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k in ("nu", "relax"):
            arr = getattr(o, k)
            for i, x in enumerate(v):
                arr[i] = int(x)
        elif k == "prec":
            o.prec = {"fp64": ADR_PREC_FP64, "mixed": ADR_PREC_MIXED}.get(v, v)
        elif k == "cycle":
            o.cycle = {"v": ADR_CYCLE_V, "k": ADR_CYCLE_K}.get(v, v)
        elif k == "advection":
            o.advection = {"upwind": ADR_ADV_UPWIND, "central": ADR_ADV_CENTRAL}.get(v, v)
        elif k == "reaction":
            o.reaction = {"numerical": ADR_REACTION_NUMERICAL, "eikonal": ADR_REACTION_EIKONAL}.get(v, v)
        else:
            setattr(o, k, v)
    return o


def two_stage_options(prec="mixed"):
    """Options of the two contexts of the two-stage solve (adr_two_stage_options)."""
    lib = load_library()
    first, second = AdrOptions(), AdrOptions()
    first.prec = {"fp64": ADR_PREC_FP64, "mixed": ADR_PREC_MIXED}.get(prec, prec)
    lib.adr_two_stage_options(ctypes.byref(first), ctypes.byref(second))
    return first, second


def solve_two_stage(first, second, q, tol=1e-6, maxit=500, tol_first=1e-2, maxit_first=5, out=None):
    """adr_solve_two_stage on two Contexts of one problem; returns (a, stats1, stats2)."""
    import torch
    a = first._new(torch.complex128) if out is None else out
    s1, s2 = AdrStats(), AdrStats()
    status = _check(first._lib.adr_solve_two_stage(first._ptr, second._ptr, _dev(q, torch.complex128),
                                                   _dev(a, torch.complex128), float(tol_first), int(maxit_first),
                                                   float(tol), int(maxit), ctypes.byref(s1), ctypes.byref(s2)),
                    second._ptr)
    d1, d2 = s1.as_dict(), s2.as_dict()
    d2["status"] = status
    return a, d1, d2


def receiver_residual_noalloc(u, idx, d, out, stream=None):
    """adr_receiver_residual_noalloc: (r, misfit) with r_k = u[idx_k] - d_k, no context and
    no allocation by the library; ``out`` (complex128, idx.numel() entries) is the caller's."""
    import torch
    lib = load_library()
    J = ctypes.c_double()
    _check(lib.adr_receiver_residual_noalloc(_dev(u, torch.complex128), _dev(idx, torch.int32),
                                             _dev(d, torch.complex128), int(idx.numel()),
                                             _dev(out, torch.complex128), ctypes.byref(J), _stream_ptr(stream)))
    return out, J.value


def eikonal(kappa2, h, src, max_sweeps=100000, stream=None):
    """adr_eikonal: first-arrival travel time (float64 tensor of kappa2's shape) from the
    source node ``src`` (NumPy axis order) by factored-eikonal sweeps on the GPU; returns
    (tau, sweeps that changed a value)."""
    import torch
    lib = load_library()
    d = kappa2.dim()
    n = (ctypes.c_int * 3)(*[kappa2.shape[d - 1 - k] if k < d else 1 for k in range(3)])
    s = (ctypes.c_int * 3)(*[int(src[d - 1 - k]) if k < d else 0 for k in range(3)])
    tau = torch.empty_like(kappa2)
    work = torch.empty(kappa2.numel() + 1, dtype=torch.float64, device=kappa2.device)
    sweeps = ctypes.c_int()
    _check(lib.adr_eikonal(d, n, float(h), _dev(kappa2, torch.float64), s, _dev(tau, torch.float64),
                           _dev(work, torch.float64), int(max_sweeps), ctypes.byref(sweeps), _stream_ptr(stream)))
    return tau, sweeps.value


def tuning_table_write(path):
    """Write the autotuner's table (adr_tuning_table_write); returns the entry count."""
    n = load_library().adr_tuning_table_write(os.fsencode(path))
    if n < 0:
        raise OSError(f"cannot write the tuning table to {path}")
    return n


def tuning_table_read(path):
    """Load a table written by tuning_table_write; returns the entry count."""
    n = load_library().adr_tuning_table_read(os.fsencode(path))
    if n < 0:
        raise OSError(f"cannot read the tuning table {path}")
    return n


def _check(status, ctx_ptr=None):
    if status != ADR_OK and status != ADR_ENOCONV:
        lib = load_library()
        msg = lib.adr_last_error(ctx_ptr)
        raise AdrError(status, (msg or b"").decode() or lib.adr_strerror(status).decode())
    return status


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    import torch
    if not t.is_cuda:
        raise ValueError("tensors must be on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def make_problem(kappa2, tau, gamma, h, omega, src, factored=True):
    """adr_problem for device tensors (NumPy axis order; reversed for the ABI).  tau=None:
    the standard Helmholtz operator (tau = 0, no factoring)."""
    import torch
    shape = tuple(kappa2.shape)
    d = len(shape)
    prob = AdrProblem()
    prob.ndim = d
    for k in range(3):
        prob.n[k] = shape[d - 1 - k] if k < d else 1
    prob.h = float(h)
    prob.omega = float(omega)
    prob.kappa2 = _dev(kappa2, torch.float64)
    prob.tau = _dev(tau, torch.float64) if tau is not None else None
    prob.gamma = _dev(gamma, torch.float64) if gamma is not None else None
    if factored and src is not None:
        for k in range(3):
            prob.src[k] = int(src[d - 1 - k]) if k < d else 0
    else:
        prob.src[0], prob.src[1], prob.src[2] = -1, 0, 0
    return prob


class Context:
    """An adr_ctx: coefficients, multigrid hierarchy and solver buffers for one source."""

    def __init__(self, kappa2, tau, gamma, h, omega, src, options=None, stream=None, factored=True, _borrowed=None):
        lib = load_library()
        self._lib = lib
        ref = tau if tau is not None else kappa2
        self.shape = tuple(ref.shape)
        self.device = ref.device
        if _borrowed is not None:   # a context owned by a Batch
            self._ptr = _borrowed
            self._owned = False
            self.options = options
            return
        prob = make_problem(kappa2, tau, gamma, h, omega, src, factored)
        self.options = options if options is not None else default_options()
        self._stream = stream
        ptr = ctypes.c_void_p()
        status = lib.adr_setup(ctypes.byref(prob), ctypes.byref(self.options), _stream_ptr(stream), ctypes.byref(ptr))
        if status != ADR_OK:
            raise AdrError(status, (lib.adr_last_error(None) or b"").decode())
        self._ptr = ptr
        self._owned = True

    def close(self):
        if getattr(self, "_ptr", None):
            if self._owned:
                self._lib.adr_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _new(self, dtype):
        import torch
        return torch.empty(self.shape, dtype=dtype, device=self.device)

    def apply(self, x, beta=0.0, out=None):
        import torch
        y = self._new(torch.complex128) if out is None else out
        _check(self._lib.adr_apply(self._ptr, float(beta), _dev(x, torch.complex128), _dev(y, torch.complex128)),
               self._ptr)
        return y

    def vcycle(self, r, out=None):
        import torch
        z = self._new(torch.complex128) if out is None else out
        _check(self._lib.adr_vcycle(self._ptr, _dev(r, torch.complex128), _dev(z, torch.complex128)), self._ptr)
        return z

    def solve(self, q, tol=1e-6, maxit=500, x0=None, out=None):
        """Returns (a, stats dict).  stats['status'] is ADR_OK or ADR_ENOCONV."""
        import torch
        a = self._new(torch.complex128) if out is None else out
        use_guess = 0
        if x0 is not None:
            a.copy_(x0)
            use_guess = 1
        st = AdrStats()
        status = _check(self._lib.adr_solve(self._ptr, _dev(q, torch.complex128), _dev(a, torch.complex128),
                                            float(tol), int(maxit), use_guess, ctypes.byref(st)), self._ptr)
        d = st.as_dict()
        d["status"] = status
        return a, d

    def solve_adjoint(self, s, tol=1e-6, maxit=500, x0=None, out=None):
        """lam with H_2up^H lam = s exp(i w tau); returns (lam, stats dict)."""
        import torch
        lam = self._new(torch.complex128) if out is None else out
        use_guess = 0
        if x0 is not None:
            lam.copy_(x0)
            use_guess = 1
        st = AdrStats()
        status = _check(self._lib.adr_solve_adjoint(self._ptr, _dev(s, torch.complex128), _dev(lam, torch.complex128),
                                                    float(tol), int(maxit), use_guess, ctypes.byref(st)), self._ptr)
        d = st.as_dict()
        d["status"] = status
        return lam, d

    def apply_adjoint(self, x, out=None):
        import torch
        y = self._new(torch.complex128) if out is None else out
        _check(self._lib.adr_apply_adjoint(self._ptr, _dev(x, torch.complex128), _dev(y, torch.complex128)),
               self._ptr)
        return y

    def grad_kappa2(self, a, lam, grad):
        """grad += -Re(conj(lam) (w^2 - i w gamma) a)  (grad: float64 tensor, accumulated)."""
        import torch
        _check(self._lib.adr_grad_kappa2(self._ptr, _dev(a, torch.complex128), _dev(lam, torch.complex128),
                                         _dev(grad, torch.float64)), self._ptr)
        return grad

    def receiver_residual(self, u, idx, d, out=None):
        """(r, misfit): r_k = u[idx_k] - d_k, misfit = 1/2 sum |r_k|^2 (idx: int32 linear indices)."""
        import torch
        n = int(idx.numel())
        r = torch.empty(n, dtype=torch.complex128, device=self.device) if out is None else out
        J = ctypes.c_double()
        _check(self._lib.adr_receiver_residual(self._ptr, _dev(u, torch.complex128), _dev(idx, torch.int32),
                                               _dev(d, torch.complex128), n, _dev(r, torch.complex128),
                                               ctypes.byref(J)), self._ptr)
        return r, J.value

    def adjoint_source(self, idx, r, out=None):
        import torch
        s = self._new(torch.complex128) if out is None else out
        _check(self._lib.adr_adjoint_source(self._ptr, _dev(idx, torch.int32), _dev(r, torch.complex128),
                                            int(idx.numel()), _dev(s, torch.complex128)), self._ptr)
        return s

    def wavefield(self, a, out=None):
        import torch
        u = self._new(torch.complex128) if out is None else out
        _check(self._lib.adr_wavefield(self._ptr, _dev(a, torch.complex128), _dev(u, torch.complex128)), self._ptr)
        return u

    def coefficients(self):
        """(g, L, c): g has one plane per axis in ABI order (axis 0 = x)."""
        import torch
        d = len(self.shape)
        g = torch.empty((d,) + self.shape, dtype=torch.float64, device=self.device)
        L = self._new(torch.float64)
        c = self._new(torch.complex128)
        _check(self._lib.adr_get_coefficients(self._ptr, _dev(g, torch.float64), _dev(L, torch.float64),
                                              _dev(c, torch.complex128)), self._ptr)
        return g, L, c

    def timer_start(self, kind, level=-1):
        kind = TIMER_KINDS.get(kind, kind)
        _check(self._lib.adr_timer_start(self._ptr, int(kind), int(level)), self._ptr)

    def timer_stop(self):
        """(total kernel ms, launches, algorithmic bytes) since timer_start."""
        ms, n, by = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
        _check(self._lib.adr_timer_stop(self._ptr, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)), self._ptr)
        return ms.value, n.value, by.value

    @property
    def num_levels(self):
        return self._lib.adr_num_levels(self._ptr)

    def level_info(self, level):
        nodes = (ctypes.c_int * 3)()
        sp = ctypes.c_int()
        _check(self._lib.adr_level_info(self._ptr, level, nodes, ctypes.byref(sp)), self._ptr)
        d = len(self.shape)
        shape = tuple(nodes[d - 1 - k] for k in range(d))
        return shape, sp.value

    def level_split(self, level):
        """Galerkin-apply variant of coarse level ``level`` >= 1 (1 or 4)."""
        sp = ctypes.c_int()
        _check(self._lib.adr_level_split(self._ptr, level, ctypes.byref(sp)), self._ptr)
        return sp.value

    def level_stencil(self, level):
        """(planes complex128 [S, *shape_l], offsets int list of (dx, dy, dz))."""
        import torch
        shape, S = self.level_info(level)
        planes = torch.empty((S,) + shape, dtype=torch.complex128, device=self.device)
        offs = (ctypes.c_int * (3 * S))()
        _check(self._lib.adr_get_level_stencil(self._ptr, level, _dev(planes, torch.complex128), offs), self._ptr)
        return planes, [tuple(offs[3 * p:3 * p + 3]) for p in range(S)]


class Batch:
    """Many shots solved together (adr_setup_batch / adr_solve_batch).  Each entry of
    ``shots`` is a dict with kappa2, tau, gamma (device tensors), h, omega, src."""

    def __init__(self, shots, options=None, nstreams=4):
        lib = load_library()
        self._lib = lib
        self.options = options if options is not None else default_options()
        probs = (AdrProblem * len(shots))()
        for i, s in enumerate(shots):
            probs[i] = make_problem(s["kappa2"], s.get("tau"), s.get("gamma"), s["h"], s["omega"], s["src"])
        self.shapes = [tuple(s["kappa2"].shape) for s in shots]
        self.device = shots[0]["kappa2"].device
        ptr = ctypes.c_void_p()
        st = lib.adr_setup_batch(len(shots), probs, ctypes.byref(self.options), int(nstreams), ctypes.byref(ptr))
        if st != ADR_OK:
            raise AdrError(st, (lib.adr_last_error(None) or b"").decode())
        self._ptr = ptr
        self.contexts = [Context(s["kappa2"], s.get("tau"), None, s["h"], s["omega"], s["src"], options=self.options,
                                 _borrowed=ctypes.c_void_p(lib.adr_batch_context(ptr, i)))
                         for i, s in enumerate(shots)]

    def solve(self, qs, outs, tol=1e-6, maxit=500):
        """Solve every shot; returns (status, list of stats dicts)."""
        import torch
        n = len(self.contexts)
        qp = (ctypes.c_void_p * n)(*[_dev(q, torch.complex128).value for q in qs])
        ap = (ctypes.c_void_p * n)(*[_dev(a, torch.complex128).value for a in outs])
        stats = (AdrStats * n)()
        st = self._lib.adr_solve_batch(self._ptr, qp, ap, float(tol), int(maxit), stats)
        if st not in (ADR_OK, ADR_ENOCONV):
            raise AdrError(st, "batch solve failed")
        return st, [s.as_dict() for s in stats]

    def groups(self):
        """Launch groups of the batch (one per grid shape, or one when merged)."""
        return int(self._lib.adr_batch_groups(self._ptr))

    def close(self):
        if getattr(self, "_ptr", None):
            for c in self.contexts:
                c.close()
            self._lib.adr_destroy_batch(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
