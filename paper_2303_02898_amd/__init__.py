"""MI355X (gfx950) maximal-entropy moment method -- Python binding.

Argument marshalling only: every step of the hot path runs in the HIP kernels
of ``libmem_mi355x.so`` (built in-tree by ``python -m paper_2303_02898_amd.build``).
PyTorch supplies device memory and the current HIP stream.  If the library is
missing, creating a :class:`Context` raises -- there is no fallback path.

Entry points mirror ``include/mem.h``: ``gauge``, ``solve`` (mem_maxent_solve),
``dual``, ``flux``, ``collide``, ``step`` and ``conserved``.
"""

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmem_mi355x.so")

ST_CONVERGED = 0x01
ST_MAXITER = 0x02
ST_STAGNATED = 0x04
ST_SHIFTED = 0x08
ST_FP64 = 0x10
ST_NONFINITE = 0x20
ST_NONREALIZABLE = 0x40
ST_LAMBDA_FAIL = 0x80
ST_MAXWELL_FLUX = 0x100
FLUX_SCHEMES = {"llf": 0, "lw": 1, "flic": 2}

PREC = {"fp32": 0, "bf16x3": 1, "fp16x3": 2}

_c_i32, _c_i64, _c_f32, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p


class MemConfig(ctypes.Structure):
    _fields_ = [("dim", _c_i32), ("n_nodes_1d", _c_i32), ("prec", _c_i32), ("reserved", _c_i32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol_grad", _c_f32), ("tol_dec", _c_f32), ("tol_grad_loose", _c_f32),
                ("max_iter", _c_i32), ("max_ls", _c_i32), ("armijo_c", _c_f32),
                ("atol", _c_f32), ("rtol", _c_f32), ("lambda0", _c_f32),
                ("lambda_mul", _c_f32), ("alpha_min", _c_f32),
                ("fp64_pivot_ratio", _c_f32), ("check_every", _c_i32), ("refine", _c_i32),
                ("beta_max", _c_f32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_cells", _c_i64), ("n_problems", _c_i32), ("collision", _c_i32),
                ("cell_offsets", _vp), ("dx", _vp), ("M_left", _vp), ("M_right", _vp),
                ("g_left", _vp), ("g_right", _vp), ("cfl", _c_f32), ("prandtl", _c_f32),
                ("mu_ref", _c_f32), ("newton_per_step", _c_i32), ("use_graph", _c_i32),
                ("iter_hist", _vp), ("flux_scheme", _c_i32), ("cond_max", _vp),
                ("status_counts", _vp)]


_lib = None


class AxiRuleStruct(ctypes.Structure):
    _fields_ = [("ux_lo", ctypes.c_double), ("ux_hi", ctypes.c_double), ("ur_hi", ctypes.c_double),
                ("blocks_x", _c_i32), ("blocks_r", _c_i32), ("order", _c_i32), ("reserved", _c_i32)]


class AxiShockStruct(ctypes.Structure):
    _fields_ = [("n_cells", _c_i32), ("dx", _c_f32), ("cfl", _c_f32), ("prandtl", _c_f32),
                ("mu_ref", _c_f32), ("ghost_left", _c_f32 * 3), ("ghost_right", _c_f32 * 3),
                ("scheme", _c_i32), ("use_graph", _c_i32), ("cond_max", _vp)]


class AxiBatchStruct(ctypes.Structure):
    _fields_ = [("n_cells", _c_i64), ("n_problems", _c_i32), ("scheme", _c_i32),
                ("cell_offsets", _vp), ("dx", _vp), ("ghosts", _vp), ("cfl", _c_f32),
                ("prandtl", _c_f32), ("mu_ref", _c_f32), ("use_graph", _c_i32),
                ("cond_max", _vp)]


class Tuning(ctypes.Structure):
    _fields_ = [("dir_waves", _c_i32), ("split_want", _c_i32), ("tuned_ms", ctypes.c_double),
                ("solver", _c_i32), ("wave_max_cells", _c_i32), ("wave_per_cu", _c_i32),
                ("asm_waves", _c_i32), ("cached", _c_i32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def load_library():
    """Load libmem_mi355x.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with "
                           "`python -m paper_2303_02898_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, E = _vp, ctypes.c_int
    sig = {
        "mem_create": ([ctypes.POINTER(MemConfig), ctypes.POINTER(_vp)], E),
        "mem_destroy": ([P], E),
        "mem_reserve": ([P, _c_i64, _c_i32], E),
        "mem_strerror": ([E], ctypes.c_char_p),
        "mem_last_error": ([P], ctypes.c_char_p),
        "mem_solve_opts_default": ([ctypes.POINTER(SolveOpts)], None),
        "mem_n_basis": ([P], _c_i32),
        "mem_n_nodes": ([P], _c_i32),
        "mem_copy_table": ([P, _c_i32, P, _c_i64, ctypes.POINTER(_c_i64)], E),
        "mem_host_table": ([_c_i32, _c_i32, _c_i32, P, _c_i64, ctypes.POINTER(_c_i64)], E),
        "mem_gauge": ([P, _c_i64, P, P, P, P], E),
        "mem_maxent_solve": ([P, _c_i64, P, P, ctypes.POINTER(SolveOpts), P, P, P, P], E),
        "mem_maxent_solve_noalloc": ([P, _c_i64, P, P, ctypes.POINTER(SolveOpts), P, P, P, P], E),
        "mem_dual": ([P, _c_i64, P, P, P, P, P], E),
        "mem_moment_residual": ([P, _c_i64, P, P, P, P], E),
        "mem_flux": ([P, _c_i64, P, P, P, P, P], E),
        "mem_collide": ([P, _c_i64, P, P, _c_f32, _c_f32, _c_f32, P], E),
        "mem_step": ([P, ctypes.POINTER(Batch), P, P, P, P, P, _c_i32,
                      ctypes.POINTER(SolveOpts), P, P], E),
        "mem_conserved": ([P, ctypes.POINTER(Batch), P, P, P, P], E),
        "mem_autotune": ([P, _c_i64, P, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(Tuning),
                          P], E),
        "mem_get_tuning": ([P, ctypes.POINTER(Tuning)], E),
        "mem_tuning_cache_clear": ([], None),
        "mem_set_tuning": ([P, ctypes.POINTER(Tuning)], E),
        "mem_axi_domain": ([ctypes.c_double] * 4 + [_c_i32] * 3 + [P], E),
        "mem_axi_rule_nodes": ([ctypes.POINTER(AxiRuleStruct)], _c_i64),
        "mem_axi_host_rule": ([ctypes.POINTER(AxiRuleStruct), P, P, P, _c_i64], E),
        "mem_axi_create": ([ctypes.POINTER(AxiRuleStruct), ctypes.POINTER(_vp)], E),
        "mem_axi_destroy": ([P], E),
        "mem_axi_n_nodes": ([P], _c_i64),
        "mem_axi_solve": ([P, _c_i64, P, P, P, ctypes.POINTER(SolveOpts), P, P, P, P], E),
        "mem_axi_moments": ([P, _c_i64, P, P, P, P, P], E),
        "mem_axi_moments_noncanonical": ([P, _c_i64, P, P, P, P], E),
        "mem_axi_gauge": ([_c_i64, P, P, P, P], E),
        "mem_axi_speeds": ([P, _c_i64, P, P, P, P], E),
        "mem_axi_reserve": ([P, _c_i64], E),
        "mem_axi_reserve_batch": ([P, _c_i64, _c_i32], E),
        "mem_axi_step_batch": ([P, ctypes.POINTER(AxiBatchStruct), P, P, P, P, P, _c_i32,
                                ctypes.POINTER(SolveOpts), P, _vp], E),
        "mem_axi_step": ([P, ctypes.POINTER(AxiShockStruct), P, P, P, P, P, _c_i32,
                          ctypes.POINTER(SolveOpts), P, P], E),
        "mem_profile_enable": ([P, _c_i32], E),
        "mem_profile_read": ([P, _c_i32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(_c_i64)], E),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def tuning_cache_clear():
    """Forget every cached autotune result (the next autotune times again)."""
    load_library().mem_tuning_cache_clear()


def host_table(dim, n_nodes_1d, which):
    """FP64 table built by the library's host code (no device needed)."""
    import numpy as np
    lib = load_library()
    wid = {"nodes": 0, "weights": 1, "phi": 2, "logw": 3}[which]
    tot = _c_i64()
    err = lib.mem_host_table(dim, n_nodes_1d, wid, None, 0, ctypes.byref(tot))
    if err != 0:
        raise MemError(f"mem_host_table: {lib.mem_strerror(err).decode()}")
    out = np.empty(tot.value, dtype=np.float64)
    lib.mem_host_table(dim, n_nodes_1d, wid, out.ctypes.data, tot.value, None)
    K = 35 if dim == 3 else 5
    if which == "nodes":
        return out.reshape(-1, dim)
    if which == "phi":
        return out.reshape(-1, K)
    return out


def default_opts(**kw):
    lib = load_library()
    o = SolveOpts()
    lib.mem_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t, dtype=None, shape_tail=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (n, {shape_tail})")
    del torch
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class MemError(RuntimeError):
    pass


class Context:
    """A library context: quadrature/basis tables on the current device plus workspace."""

    def __init__(self, dim=3, n_nodes_1d=12, prec="fp32"):
        self._lib = load_library()
        cfg = MemConfig(dim, n_nodes_1d, PREC[prec] if isinstance(prec, str) else int(prec), 0)
        h = _vp()
        err = self._lib.mem_create(ctypes.byref(cfg), ctypes.byref(h))
        if err != 0:
            raise MemError(f"mem_create: {self._lib.mem_strerror(err).decode()}")
        self._h = h
        self.dim = dim
        self.n_nodes_1d = n_nodes_1d
        self.K = self._lib.mem_n_basis(h)
        self.Q = self._lib.mem_n_nodes(h)
        self.G = 2 if dim == 1 else 3

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, err, what):
        if err != 0:
            detail = self._lib.mem_last_error(self._h).decode()
            raise MemError(f"{what}: {self._lib.mem_strerror(err).decode()} ({detail})")

    def autotune(self, M, beta_init, opts=None, stream=None):
        """Time solves of this batch over the launch candidates; keep the fastest."""
        import torch
        work = torch.empty_like(beta_init)
        t = Tuning()
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_autotune(self._h, M.shape[0], _ptr(M, torch.float32, (self.K,), "M"),
                                           _ptr(beta_init, torch.float32, (self.K,), "beta_init"),
                                           work.data_ptr(), o, ctypes.byref(t), _stream(stream)),
                    "mem_autotune")
        return t.as_dict()

    def tuning(self):
        t = Tuning()
        self._check(self._lib.mem_get_tuning(self._h, ctypes.byref(t)), "mem_get_tuning")
        return t.as_dict()

    def set_tuning(self, dir_waves=4, split_want=512, solver=1, wave_max_cells=0, wave_per_cu=12,
                   asm_waves=4):
        t = Tuning(int(dir_waves), int(split_want), 0.0, int(solver), int(wave_max_cells),
                   int(wave_per_cu), int(asm_waves), 0)
        self._check(self._lib.mem_set_tuning(self._h, ctypes.byref(t)), "mem_set_tuning")

    def reserve(self, max_cells, max_problems=0):
        self._check(self._lib.mem_reserve(self._h, int(max_cells), int(max_problems)), "mem_reserve")

    def table(self, which):
        """Host FP64 table: 'nodes' (Q, dim), 'weights' (Q,), 'phi' (Q, K)."""
        import numpy as np
        wid = {"nodes": 0, "weights": 1, "phi": 2}[which]
        tot = _c_i64()
        self._check(self._lib.mem_copy_table(self._h, wid, None, 0, ctypes.byref(tot)), "mem_copy_table")
        out = np.empty(tot.value, dtype=np.float64)
        self._check(self._lib.mem_copy_table(self._h, wid, out.ctypes.data, tot.value, None),
                    "mem_copy_table")
        if which == "nodes":
            return out.reshape(-1, self.dim)
        if which == "phi":
            return out.reshape(-1, self.K)
        return out

    def profile(self, enable=True):
        """Enable (and clear) or disable HIP-event timing of the solver kernels."""
        self._check(self._lib.mem_profile_enable(self._h, 1 if enable else 0), "mem_profile_enable")

    def profile_read(self, kernel):
        """(total ms, launches) for kernel 'assemble', 'direction' or 'lse'."""
        kid = {"assemble": 0, "direction": 1, "lse": 2, "wave": 3}[kernel]
        ms, cnt = ctypes.c_double(), _c_i64()
        self._check(self._lib.mem_profile_read(self._h, kid, ctypes.byref(ms), ctypes.byref(cnt)),
                    "mem_profile_read")
        return ms.value, cnt.value

    # ---- hot path -------------------------------------------------------------------
    def gauge(self, M, beta, g, stream=None):
        import torch
        n = M.shape[0]
        self._check(self._lib.mem_gauge(
            self._h, n, _ptr(M, torch.float32, (self.K,), "M"),
            _ptr(beta, torch.float32, (self.K,), "beta"), _ptr(g, torch.float32, (self.G,), "g"),
            _stream(stream)), "mem_gauge")

    def solve(self, M, beta, opts=None, iters=None, resid=None, status=None, stream=None):
        import torch
        n = M.shape[0]
        dev = M.device
        if iters is None:
            iters = torch.zeros(n, dtype=torch.int32, device=dev)
        if resid is None:
            resid = torch.zeros(n, dtype=torch.float32, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_maxent_solve(
            self._h, n, _ptr(M, torch.float32, (self.K,), "M"),
            _ptr(beta, torch.float32, (self.K,), "beta"), o, _ptr(iters, torch.int32),
            _ptr(resid, torch.float32), _ptr(status, torch.int32), _stream(stream)),
            "mem_maxent_solve")
        return iters, resid, status

    def solve_noalloc(self, M, beta, opts=None, iters=None, resid=None, status=None,
                      stream=None):
        """mem_maxent_solve_noalloc: the same solve on the library's static device
        scratch (at most 8192 cells per call); the output tensors must be given
        by callers that cannot allocate."""
        import torch
        n = M.shape[0]
        dev = M.device
        if iters is None:
            iters = torch.zeros(n, dtype=torch.int32, device=dev)
        if resid is None:
            resid = torch.zeros(n, dtype=torch.float32, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_maxent_solve_noalloc(
            self._h, n, _ptr(M, torch.float32, (self.K,), "M"),
            _ptr(beta, torch.float32, (self.K,), "beta"), o, _ptr(iters, torch.int32),
            _ptr(resid, torch.float32), _ptr(status, torch.int32), _stream(stream)),
            "mem_maxent_solve_noalloc")
        return iters, resid, status

    def dual(self, beta, stream=None):
        import torch
        n = beta.shape[0]
        dev = beta.device
        logZ = torch.empty(n, dtype=torch.float32, device=dev)
        E = torch.empty(n, self.K, dtype=torch.float32, device=dev)
        H = torch.empty(n, self.K - 1, self.K - 1, dtype=torch.float32, device=dev)
        self._check(self._lib.mem_dual(self._h, n, _ptr(beta, torch.float32, (self.K,), "beta"),
                                       logZ.data_ptr(), E.data_ptr(), H.data_ptr(),
                                       _stream(stream)), "mem_dual")
        return logZ, E, H

    def moment_residual(self, M, beta, stream=None):
        """Per-moment residual G[n][K] (G_k = E[phi_k]/E[phi_0] - M_k/M_0), compensated."""
        import torch
        n = beta.shape[0]
        G = torch.empty(n, self.K, dtype=torch.float32, device=beta.device)
        self._check(self._lib.mem_moment_residual(
            self._h, n, _ptr(M, torch.float32, (self.K,), "M"),
            _ptr(beta, torch.float32, (self.K,), "beta"), G.data_ptr(), _stream(stream)),
            "mem_moment_residual")
        return G

    def flux(self, beta, g, want_lam=True, stream=None):
        import torch
        n = beta.shape[0]
        F = torch.empty(n, self.K, dtype=torch.float32, device=beta.device)
        lam = torch.empty(n, 2, dtype=torch.float32, device=beta.device) if want_lam else None
        self._check(self._lib.mem_flux(self._h, n, _ptr(beta, torch.float32, (self.K,), "beta"),
                                       _ptr(g, torch.float32, (3,), "g"), F.data_ptr(),
                                       lam.data_ptr() if lam is not None else None,
                                       _stream(stream)), "mem_flux")
        return F, lam

    def collide(self, M, g, h, prandtl=2.0 / 3.0, mu_ref=0.7978845608028654, stream=None):
        import torch
        self._check(self._lib.mem_collide(self._h, M.shape[0], _ptr(M, torch.float32, (self.K,), "M"),
                                          _ptr(g, torch.float32, (3,), "g"), float(h),
                                          float(prandtl), float(mu_ref), _stream(stream)),
                    "mem_collide")

    def step(self, batch, M, beta, g, t, dt, n_steps, opts=None, status=None, stream=None):
        import torch
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_step(
            self._h, ctypes.byref(batch.struct), _ptr(M, torch.float32, (self.K,), "M"),
            _ptr(beta, torch.float32, (self.K,), "beta"), _ptr(g, torch.float32, (3,), "g"),
            _ptr(t, torch.float32), _ptr(dt, torch.float32), int(n_steps), o,
            _ptr(status, torch.int32) if status is not None else None, _stream(stream)), "mem_step")

    def conserved(self, batch, M, g, stream=None):
        import torch
        out = torch.zeros(batch.n_problems, 3, dtype=torch.float64, device=M.device)
        self._check(self._lib.mem_conserved(self._h, ctypes.byref(batch.struct),
                                            _ptr(M, torch.float32, (self.K,), "M"),
                                            _ptr(g, torch.float32, (3,), "g"), out.data_ptr(),
                                            _stream(stream)), "mem_conserved")
        return out


def axi_domain(v_minus, T_minus, v_plus, T_plus, n_a, n_b, n_r):
    """Integration box (a_x, b_x, b_r) of the normal-shock set-up (host)."""
    lib = load_library()
    box = (ctypes.c_double * 3)()
    err = lib.mem_axi_domain(v_minus, T_minus, v_plus, T_plus, n_a, n_b, n_r, box)
    if err != 0:
        raise MemError(f"mem_axi_domain: {lib.mem_strerror(err).decode()}")
    return tuple(box)


def _axi_rule(ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order):
    return AxiRuleStruct(ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order, 0)


def axi_host_rule(ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order):
    """FP64 nodes (ux, ur, logw) of a block-wise Gauss--Legendre box, built by
    the library's host code (no device needed)."""
    import numpy as np
    lib = load_library()
    r = _axi_rule(ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order)
    P = lib.mem_axi_rule_nodes(ctypes.byref(r))
    if P < 0:
        raise MemError("mem_axi_rule_nodes: invalid rule")
    ux, ur, lw = (np.empty(P, dtype=np.float64) for _ in range(3))
    err = lib.mem_axi_host_rule(ctypes.byref(r), ux.ctypes.data, ur.ctypes.data, lw.ctypes.data, P)
    if err != 0:
        raise MemError(f"mem_axi_host_rule: {lib.mem_strerror(err).decode()}")
    return dict(ux=ux, ur=ur, logw=lw)


class AxiRule:
    """The paper's nine-statistic discretisation: a block-wise Gauss--Legendre
    box fixed in physical velocity, on the current device."""

    K = 9

    def __init__(self, ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order):
        self._lib = load_library()
        r = _axi_rule(ux_lo, ux_hi, ur_hi, blocks_x, blocks_r, order)
        h = _vp()
        err = self._lib.mem_axi_create(ctypes.byref(r), ctypes.byref(h))
        if err != 0:
            raise MemError(f"mem_axi_create: {self._lib.mem_strerror(err).decode()}")
        self._h = h
        self.n_nodes = int(self._lib.mem_axi_n_nodes(h))

    def close(self):
        if self._h:
            self._lib.mem_axi_destroy(self._h)
            self._h = None

    def _check(self, err, what):
        if err != 0:
            raise MemError(f"{what}: {self._lib.mem_strerror(err).decode()}")

    def solve(self, M, g, beta, opts=None, iters=None, resid=None, status=None, stream=None):
        import torch
        n = M.shape[0]
        dev = M.device
        if iters is None:
            iters = torch.zeros(n, dtype=torch.int32, device=dev)
        if resid is None:
            resid = torch.zeros(n, dtype=torch.float32, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_axi_solve(
            self._h, n, _ptr(M, torch.float32, (9,), "M"), _ptr(g, torch.float32, (3,), "g"),
            _ptr(beta, torch.float32, (9,), "beta"), o, _ptr(iters, torch.int32),
            _ptr(resid, torch.float32), _ptr(status, torch.int32), _stream(stream)), "mem_axi_solve")
        return iters, resid, status

    def reserve(self, n_cells, n_problems=1):
        """Size the time-step workspace (step calls then allocate nothing)."""
        self._check(self._lib.mem_axi_reserve_batch(self._h, int(n_cells), int(n_problems)),
                    "mem_axi_reserve_batch")

    def step_batch(self, M, beta, g, t, dt, cell_offsets, dx, ghosts, n_steps=1, cfl=0.5,
                   prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi), opts=None, status=None,
                   scheme="llf", use_graph=False, cond_max=None, stream=None):
        """Alg. 2 time steps of a ragged batch of shock problems (n_steps = 0:
        set-up only).  cell_offsets: device int64 [P + 1]; dx: device [P];
        ghosts: device [P, 6] = left (n, v, T), right (n, v, T); t, dt: device [P]."""
        import torch
        P = cell_offsets.shape[0] - 1
        n = M.shape[0]
        if dx.shape != (P,) or ghosts.shape != (P, 6) or t.shape != (P,) or dt.shape != (P,):
            raise ValueError("dx, t, dt must be [P] and ghosts [P, 6]")
        b = AxiBatchStruct(n, P, FLUX_SCHEMES[scheme], _ptr(cell_offsets, torch.int64, name="cell_offsets"),
                           _ptr(dx, torch.float32, name="dx"),
                           _ptr(ghosts, torch.float32, (6,), "ghosts"), cfl, prandtl, mu_ref,
                           1 if use_graph else 0,
                           _ptr(cond_max, torch.float32, name="cond_max"))
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_axi_step_batch(
            self._h, ctypes.byref(b), _ptr(M, torch.float32, (9,), "M"),
            _ptr(beta, torch.float32, (9,), "beta"), _ptr(g, torch.float32, (3,), "g"),
            _ptr(t, torch.float32), _ptr(dt, torch.float32), n_steps, o,
            _ptr(status, torch.int32) if status is not None else None, _stream(stream)),
            "mem_axi_step_batch")

    def step(self, M, beta, g, t, dt, dx, left, right, n_steps=1, cfl=0.5,
             prandtl=2.0 / 3.0, mu_ref=math.sqrt(2.0 / math.pi), opts=None, status=None,
             scheme="llf", use_graph=False, cond_max=None, stream=None):
        """Alg. 2 time steps of one shock problem (n_steps = 0: set-up only).
        left/right: ghost (n, v, T); t, dt: one-element device tensors;
        use_graph: replay a captured step; cond_max: one-element device tensor,
        the running max of the in-kernel lower bound of cond(H)."""
        import torch
        n = M.shape[0]
        pb = AxiShockStruct(n, dx, cfl, prandtl, mu_ref, (_c_f32 * 3)(*left),
                            (_c_f32 * 3)(*right), FLUX_SCHEMES[scheme], 1 if use_graph else 0,
                            _ptr(cond_max, torch.float32, name="cond_max"))
        o = ctypes.byref(opts) if opts is not None else None
        self._check(self._lib.mem_axi_step(
            self._h, ctypes.byref(pb), _ptr(M, torch.float32, (9,), "M"),
            _ptr(beta, torch.float32, (9,), "beta"), _ptr(g, torch.float32, (3,), "g"),
            _ptr(t, torch.float32), _ptr(dt, torch.float32), n_steps, o,
            _ptr(status, torch.int32) if status is not None else None, _stream(stream)),
            "mem_axi_step")

    def speeds(self, beta, g, stream=None):
        """(min, max) characteristic speed per cell in physical velocity."""
        import torch
        n = beta.shape[0]
        lam = torch.empty(n, 2, dtype=torch.float32, device=beta.device)
        self._check(self._lib.mem_axi_speeds(
            self._h, n, _ptr(beta, torch.float32, (9,), "beta"), _ptr(g, torch.float32, (3,), "g"),
            lam.data_ptr(), _stream(stream)), "mem_axi_speeds")
        return lam

    def gauge(self, M, beta, g, stream=None):
        """Move M (and beta, if given) into the Hermite gauge of M; g updated."""
        import torch
        n = M.shape[0]
        self._check(self._lib.mem_axi_gauge(
            n, _ptr(M, torch.float32, (9,), "M"),
            _ptr(beta, torch.float32, (9,), "beta") if beta is not None else None,
            _ptr(g, torch.float32, (3,), "g"), _stream(stream)), "mem_axi_gauge")

    def moments_noncanonical(self, alpha, g, stream=None):
        """Moments of f = exp(alpha_0 + alpha_i phi_i), plain FP32 sums (no shift)."""
        import torch
        n = alpha.shape[0]
        M = torch.empty(n, 9, dtype=torch.float32, device=alpha.device)
        self._check(self._lib.mem_axi_moments_noncanonical(
            self._h, n, _ptr(alpha, torch.float32, (9,), "alpha"),
            _ptr(g, torch.float32, (3,), "g"), M.data_ptr(), _stream(stream)),
            "mem_axi_moments_noncanonical")
        return M

    def moments(self, beta, g, want_flux=True, stream=None):
        import torch
        n = beta.shape[0]
        M = torch.empty(n, 9, dtype=torch.float32, device=beta.device)
        F = torch.empty(n, 9, dtype=torch.float32, device=beta.device) if want_flux else None
        self._check(self._lib.mem_axi_moments(
            self._h, n, _ptr(beta, torch.float32, (9,), "beta"), _ptr(g, torch.float32, (3,), "g"),
            M.data_ptr(), F.data_ptr() if F is not None else None, _stream(stream)),
            "mem_axi_moments")
        return M, F


class ShockBatch:
    """Device-side description of a ragged batch of 1D shock problems (mem_batch_t)."""

    def __init__(self, offsets, dx, M_left, M_right, g_left, g_right, device="cuda",
                 cfl=0.5, prandtl=2.0 / 3.0, mu_ref=0.7978845608028654, collision=1,
                 newton_per_step=8, use_graph=False, iter_hist=None, flux_scheme="llf",
                 cond_max=None, status_counts=None):
        import torch
        if flux_scheme not in FLUX_SCHEMES:
            raise ValueError(f"flux_scheme must be one of {sorted(FLUX_SCHEMES)}")
        f32 = dict(dtype=torch.float32, device=device)
        self.offsets = torch.as_tensor(offsets, dtype=torch.int64, device=device).contiguous()
        self.n_problems = int(self.offsets.numel() - 1)
        self.n_cells = int(self.offsets[-1].item())
        self.dx = torch.as_tensor(dx, **f32).reshape(self.n_problems).contiguous()
        self.M_left = torch.as_tensor(M_left, **f32).reshape(self.n_problems, 35).contiguous()
        self.M_right = torch.as_tensor(M_right, **f32).reshape(self.n_problems, 35).contiguous()
        self.g_left = torch.as_tensor(g_left, **f32).reshape(self.n_problems, 3).contiguous()
        self.g_right = torch.as_tensor(g_right, **f32).reshape(self.n_problems, 3).contiguous()
        self.struct = Batch(self.n_cells, self.n_problems, int(collision), self.offsets.data_ptr(),
                            self.dx.data_ptr(), self.M_left.data_ptr(), self.M_right.data_ptr(),
                            self.g_left.data_ptr(), self.g_right.data_ptr(), float(cfl),
                            float(prandtl), float(mu_ref), int(newton_per_step),
                            int(bool(use_graph)), None, FLUX_SCHEMES[flux_scheme])
        # iteration histogram (device int64 [newton_per_step + 1]), accumulated by mem_step
        self.iter_hist = None
        if iter_hist is not None:
            if (iter_hist.dtype != torch.int64 or not iter_hist.is_contiguous()
                    or iter_hist.numel() != int(newton_per_step) + 1 or not iter_hist.is_cuda):
                raise ValueError("iter_hist must be a contiguous device int64 tensor of "
                                 "newton_per_step + 1 bins")
            self.iter_hist = iter_hist
            self.struct.iter_hist = iter_hist.data_ptr()
        # conditioning monitor (device float32 [n_problems]), accumulated by mem_step
        self.cond_max = None
        if cond_max is not None:
            if (cond_max.dtype != torch.float32 or not cond_max.is_contiguous()
                    or cond_max.numel() != self.n_problems or not cond_max.is_cuda):
                raise ValueError("cond_max must be a contiguous device float32 tensor of "
                                 "n_problems entries")
            self.cond_max = cond_max
            self.struct.cond_max = cond_max.data_ptr()
        # cell-steps by status bit (device int64 [9]), accumulated by mem_step
        self.status_counts = None
        if status_counts is not None:
            if (status_counts.dtype != torch.int64 or not status_counts.is_contiguous()
                    or status_counts.numel() != 9 or not status_counts.is_cuda):
                raise ValueError("status_counts must be a contiguous device int64 tensor of 9 "
                                 "entries")
            self.status_counts = status_counts
            self.struct.status_counts = status_counts.data_ptr()
