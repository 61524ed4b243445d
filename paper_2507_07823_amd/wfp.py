"""Python binding of libwfp (include/wfp.h): argument marshalling only.

Every step of the march runs in the HIP library; this module never computes
any part of the method.  Device arrays are torch tensors on the current CUDA
(HIP) device; problem data is passed as host numpy arrays and copied by the
library.  Importing this module does not touch the GPU; ``load_library``
raises if libwfp.so has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwfp.so")

WFP_OK = 0
WFP_EINVAL = -1
WFP_EDOMAIN = -2
WFP_ENOMEM = -3
WFP_EHIP = -4
WFP_ESTATE = -5
WFP_ENONFINITE = -6
PERIODIC = 0
FREE_SPACE = 1
STAGES = ("spread", "fft_fwd", "modes", "rbc", "fft_inv", "local", "solve", "receivers")

_c_dp = ctypes.POINTER(ctypes.c_double)


class Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("x", _c_dp), ("beta", _c_dp), ("boundary", ctypes.c_int32),
                ("n_packets", ctypes.c_int32), ("packets", _c_dp), ("R", ctypes.c_int64),
                ("x_recv", _c_dp)]


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("eps_window", ctypes.c_double), ("gamma", ctypes.c_double),
                ("W", ctypes.c_int32), ("p", ctypes.c_int32), ("K", ctypes.c_int64),
                ("n_gl_local", ctypes.c_int32), ("n_gl_pq", ctypes.c_int32), ("rbc_period", ctypes.c_int32),
                ("nufft_width", ctypes.c_int32), ("solve_iters", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32), ("overlap_cus", ctypes.c_int32),
                ("local_mode", ctypes.c_int32), ("check_finite", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("R", ctypes.c_int64), ("K", ctypes.c_int64), ("n_fine", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_pairs_recv", ctypes.c_int64), ("level", ctypes.c_int64),
                ("W", ctypes.c_int32), ("p", ctypes.c_int32), ("m_max", ctypes.c_int32),
                ("n_gl_local", ctypes.c_int32), ("rbc_period", ctypes.c_int32), ("nufft_width", ctypes.c_int32),
                ("solve_iters", ctypes.c_int32), ("boundary", ctypes.c_int32), ("dt", ctypes.c_double),
                ("delta", ctypes.c_double), ("b", ctypes.c_double), ("solve_contraction", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("n_weights_nonzero", ctypes.c_int64),
                ("n_weights_stored", ctypes.c_int64), ("solve_mode", ctypes.c_int32), ("overlap_cus", ctypes.c_int32),
                ("local_mode", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n_weights_lag1", ctypes.c_int64),
                ("n_solve_tiles", ctypes.c_int32), ("n_direct_tiles", ctypes.c_int32),
                ("sweep_wave", ctypes.c_int32), ("reserved2", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library():
    """Load libwfp.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libwfp.so not built ({LIB_PATH}); run python -m paper_2507_07823_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.wfp_plan_create.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    lib.wfp_plan_create.restype = ctypes.c_int32
    lib.wfp_plan_destroy.argtypes = [vp]
    lib.wfp_plan_destroy.restype = None
    lib.wfp_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.wfp_plan_info.restype = ctypes.c_int32
    lib.wfp_run.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, vp]
    lib.wfp_run.restype = ctypes.c_int32
    lib.wfp_run_noalloc.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, vp]
    lib.wfp_run_noalloc.restype = ctypes.c_int32
    lib.wfp_run_driven.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_int64, vp]
    lib.wfp_run_driven.restype = ctypes.c_int32
    lib.wfp_local_part.argtypes = [vp, vp]
    lib.wfp_local_part.restype = ctypes.c_int32
    lib.wfp_adjoint.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    lib.wfp_adjoint.restype = ctypes.c_int32
    lib.wfp_get_state.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, vp]
    lib.wfp_get_state.restype = ctypes.c_int32
    lib.wfp_set_state.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
    lib.wfp_set_state.restype = ctypes.c_int32
    lib.wfp_set_profiling.argtypes = [vp, ctypes.c_int32]
    lib.wfp_set_profiling.restype = ctypes.c_int32
    lib.wfp_get_profile.argtypes = [vp, _c_dp, ctypes.POINTER(ctypes.c_int64)]
    lib.wfp_get_profile.restype = ctypes.c_int32
    lib.wfp_reset.argtypes = [vp]
    lib.wfp_reset.restype = ctypes.c_int32
    lib.wfp_plan_autotune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.wfp_plan_autotune.restype = ctypes.c_int32
    lib.wfp_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Problem), ctypes.POINTER(Params), vp,
                                     ctypes.POINTER(vp)]
    lib.wfp_batch_create.restype = ctypes.c_int32
    lib.wfp_batch_run.argtypes = [vp, ctypes.c_int64, vp, vp]
    lib.wfp_batch_run.restype = ctypes.c_int32
    lib.wfp_batch_set_levels.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.wfp_batch_set_levels.restype = ctypes.c_int32
    lib.wfp_batch_reset.argtypes = [vp]
    lib.wfp_batch_reset.restype = ctypes.c_int32
    lib.wfp_batch_autotune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.wfp_batch_autotune.restype = ctypes.c_int32
    lib.wfp_batch_set_shape.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.wfp_batch_set_shape.restype = ctypes.c_int32
    lib.wfp_batch_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.wfp_batch_size.restype = ctypes.c_int32
    lib.wfp_batch_plan.argtypes = [vp, ctypes.c_int32]
    lib.wfp_batch_plan.restype = vp
    lib.wfp_batch_destroy.argtypes = [vp]
    lib.wfp_batch_destroy.restype = None
    lib.wfp_status_string.argtypes = [ctypes.c_int32]
    lib.wfp_status_string.restype = ctypes.c_char_p
    lib.wfp_last_error.argtypes = []
    lib.wfp_last_error.restype = ctypes.c_char_p
    lib.wfp_abi_version.argtypes = []
    lib.wfp_abi_version.restype = ctypes.c_int32
    _lib = lib
    return lib


class WFPError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"wfp status {status}: {message}")
        self.status = status


def _check(status):
    if status != WFP_OK:
        lib = load_library()
        raise WFPError(status, lib.wfp_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dbl(a):
    return a.ctypes.data_as(_c_dp) if a is not None and a.size else None


def make_params(dt, **kw):
    prm = Params()
    prm.dt = float(dt)
    for k, v in kw.items():
        if not hasattr(prm, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(prm, k, v)
    return prm


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _fill_problem(pr, problem, keep):
    x = np.ascontiguousarray(problem["x"], dtype=np.float64)
    beta = np.ascontiguousarray(problem["beta"], dtype=np.float64)
    packets = np.ascontiguousarray(np.atleast_2d(problem["packets"]), dtype=np.float64)
    xr = problem.get("x_recv")
    xr = np.zeros(0) if xr is None else np.ascontiguousarray(xr, dtype=np.float64)
    keep += [x, beta, packets, xr]
    pr.M = x.size
    pr.x = _dbl(x)
    pr.beta = _dbl(beta)
    pr.boundary = int(problem.get("boundary", PERIODIC))
    pr.n_packets = packets.shape[0]
    pr.packets = _dbl(packets)
    pr.R = xr.size
    pr.x_recv = _dbl(xr)


class Plan:
    """A WFP plan on the current device (all precompute done at construction).

    problem: dict with x, beta, packets (n, 5), boundary, x_recv (optional)
    dt and keyword parameters as in ``wfp_params``.
    """

    def __init__(self, problem, dt, stream=None, **params):
        lib = load_library()
        self._lib = lib
        self._keep = []
        self._owned = True
        pr = Problem()
        _fill_problem(pr, problem, self._keep)
        prm = make_params(dt, **params)
        self._stream = stream if stream is not None else _current_stream()
        h = ctypes.c_void_p()
        _check(lib.wfp_plan_create(ctypes.byref(pr), ctypes.byref(prm), self._stream, ctypes.byref(h)))
        self._h = h
        self.info = self.query_info()

    def query_info(self):
        info = Info()
        _check(self._lib.wfp_plan_info(self._h, ctypes.byref(info)))
        return info.as_dict()

    @property
    def level(self):
        return self.query_info()["level"]

    def run(self, n_steps, sigma_out=None, save_every=1, u_recv_out=None):
        """March n_steps levels into caller-provided device tensors (float64)."""
        for t in (sigma_out, u_recv_out):
            if t is not None:
                assert t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous() and t.is_cuda
        if sigma_out is not None:
            rows = (n_steps + save_every - 1) // save_every
            assert sigma_out.numel() >= rows * self.info["M"]
        if u_recv_out is not None:
            assert u_recv_out.numel() >= n_steps * self.info["R"]
        _check(self._lib.wfp_run(self._h, int(n_steps), _ptr(sigma_out), int(save_every), _ptr(u_recv_out)))

    def run_noalloc(self, n_steps, sigma_out=None, save_every=1, u_recv_out=None):
        """As run(), through wfp_run_noalloc (no device allocation in the call)."""
        for t in (sigma_out, u_recv_out):
            if t is not None:
                assert t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous() and t.is_cuda
        if sigma_out is not None:
            rows = (n_steps + save_every - 1) // save_every
            assert sigma_out.numel() >= rows * self.info["M"]
        if u_recv_out is not None:
            assert u_recv_out.numel() >= n_steps * self.info["R"]
        _check(self._lib.wfp_run_noalloc(self._h, int(n_steps), _ptr(sigma_out), int(save_every),
                                         _ptr(u_recv_out)))

    def march(self, n_steps, save_every=1, receivers=True):
        """Allocate outputs and march; returns (sigma rows, receiver values or None)."""
        import torch
        M, R = self.info["M"], self.info["R"]
        rows = (n_steps + save_every - 1) // save_every
        sig = torch.empty((rows, M), dtype=torch.float64, device="cuda")
        u = torch.empty((n_steps, R), dtype=torch.float64, device="cuda") if (receivers and R) else None
        self.run(n_steps, sig, save_every, u)
        return sig, u

    def march_driven(self, g, save_every=1, receivers=True):
        """March g.shape[0] levels with caller driving data g (float64 CUDA
        tensor [n_steps][M], caller's spring order; g_j = beta_j f(x_j - t) for
        an incident wave); returns (sigma rows, receiver values or None)."""
        import torch
        assert g.dtype == torch.float64 and g.is_cuda and g.is_contiguous() and g.dim() == 2
        n_steps, M = g.shape
        assert M == self.info["M"]
        R = self.info["R"]
        rows = (n_steps + save_every - 1) // save_every
        sig = torch.empty((rows, M), dtype=torch.float64, device="cuda")
        u = torch.empty((n_steps, R), dtype=torch.float64, device="cuda") if (receivers and R) else None
        _check(self._lib.wfp_run_driven(self._h, int(n_steps), _ptr(g), _ptr(sig), int(save_every), _ptr(u)))
        return sig, u

    def local_part(self):
        """The explicit local part (lags >= 1) at every spring for the next level."""
        import torch
        out = torch.empty(self.info["M"], dtype=torch.float64, device="cuda")
        _check(self._lib.wfp_local_part(self._h, _ptr(out)))
        return out

    def gradient(self, dJdu, positions=True):
        """dJ/dbeta and dJ/dx (or None) for the levels 0..N-1 run since the
        last reset, given dJ/du at the receivers (device tensor [N][R])."""
        import torch
        assert dJdu.dtype == torch.float64 and dJdu.is_cuda and dJdu.is_contiguous() and dJdu.dim() == 2
        M = self.info["M"]
        gb = torch.empty(M, dtype=torch.float64, device="cuda")
        gx = torch.empty(M, dtype=torch.float64, device="cuda") if positions else None
        _check(self._lib.wfp_adjoint(self._h, int(dJdu.shape[0]), _ptr(dJdu), _ptr(gb), _ptr(gx)))
        return gb, gx

    def get_state(self):
        import torch
        i = self.query_info()
        M, K, W, mm = i["M"], i["K"], i["W"], i["m_max"]
        hist = torch.empty((mm, M), dtype=torch.float64, device="cuda")
        ring = torch.empty((W, K + 1, 2), dtype=torch.float64, device="cuda")
        a = torch.empty((K + 1, 2), dtype=torch.float64, device="cuda")
        da = torch.empty((K + 1, 2), dtype=torch.float64, device="cuda")
        lvl = ctypes.c_int64()
        _check(self._lib.wfp_get_state(self._h, ctypes.byref(lvl), _ptr(hist), _ptr(ring), _ptr(a), _ptr(da)))
        return dict(L=lvl.value, hist=hist, ring=ring, alpha=a, dalpha=da)

    def set_state(self, level, hist, ring, alpha, dalpha):
        for t in (hist, ring, alpha, dalpha):
            assert t.dtype.itemsize == 8 if hasattr(t.dtype, "itemsize") else True
            assert t.is_contiguous() and t.is_cuda
        _check(self._lib.wfp_set_state(self._h, int(level), _ptr(hist), _ptr(ring), _ptr(alpha), _ptr(dalpha)))

    def set_profiling(self, on=True):
        _check(self._lib.wfp_set_profiling(self._h, 1 if on else 0))

    def profile(self):
        """{stage: (total ms, launches)} from the library's HIP-event timing."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(self._lib.wfp_get_profile(self._h, ms, n))
        return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}

    def reset(self):
        _check(self._lib.wfp_reset(self._h))

    def autotune(self, trial_levels=20):
        """Time the concurrent-schedule splits from level 0, keep the fastest
        (returns its overlap_cus, -1 for one stream); leaves the plan at level 0."""
        out = ctypes.c_int32()
        _check(self._lib.wfp_plan_autotune(self._h, int(trial_levels), ctypes.byref(out)))
        self.info = self.query_info()
        return out.value

    @classmethod
    def _borrow(cls, lib, handle):
        """A non-owning view of a plan that belongs to a batch."""
        p = cls.__new__(cls)
        p._lib = lib
        p._keep = []
        p._owned = False
        p._h = ctypes.c_void_p(handle)
        p.info = p.query_info()
        return p

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and getattr(self, "_owned", True):
            self._lib.wfp_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(x, beta, incident, dt, n_steps, boundary=0, x_recv=None, save_every=1, **params):
    """One call: plan, march n_steps levels, release the plan.

    x, beta   spring positions and stiffnesses (M; numpy arrays or tensors on
              any device; the plan copies them)
    incident  packets (n, 5): rows (amp, centre, width, omega, phase) of
              f(s) = sum amp exp(-(s - centre)^2 / (2 width^2)) cos(omega (s - centre) + phase)
    boundary  0 periodic box [-pi, pi), 1 free space
    x_recv    receiver positions (R) or None
    params    plan parameters (p, W, K, local_mode, ...; see make_params)
    Returns (u_recv [n_steps][R] or None, sigma [ceil(n_steps/save_every)][M]),
    float64 CUDA tensors in the caller's spring order."""
    def host(a):
        if a is None:
            return np.zeros(0)
        if hasattr(a, "detach"):
            a = a.detach().cpu().numpy()
        return np.ascontiguousarray(a, dtype=np.float64)

    prob = dict(x=host(x), beta=host(beta), packets=np.atleast_2d(host(incident)), boundary=int(boundary),
                x_recv=host(x_recv))
    plan = Plan(prob, dt, **params)
    try:
        sig, u = plan.march(n_steps, save_every)
    finally:
        plan.close()
    return u, sig


class Batch:
    """Independent periodic problems marched in lockstep (wfp_batch_*).

    problems: list of dicts as for Plan (receivers allowed), dts: list of time
    steps, keyword parameters shared by every instance, per_instance: optional
    list of per-instance parameter dicts.
    """

    def __init__(self, problems, dts, stream=None, per_instance=None, **params):
        lib = load_library()
        self._lib = lib
        self._keep = []
        n = len(problems)
        probs = (Problem * n)()
        pars = (Params * n)()
        for i, (pb, dt) in enumerate(zip(problems, dts)):
            _fill_problem(probs[i], pb, self._keep)
            kw = dict(params)
            if per_instance is not None:
                kw.update(per_instance[i])
            pars[i] = make_params(dt, **kw)
        self._keep += [probs, pars]
        self.n = n
        self._stream = stream if stream is not None else _current_stream()
        h = ctypes.c_void_p()
        _check(lib.wfp_batch_create(n, probs, pars, self._stream, ctypes.byref(h)))
        self._h = h
        self.sizes = [int(np.asarray(p["x"]).size) for p in problems]
        self.receivers = [int(np.asarray(p.get("x_recv", np.zeros(0))).size) for p in problems]

    @property
    def level(self):
        lvl = ctypes.c_int64()
        _check(self._lib.wfp_batch_size(self._h, None, ctypes.byref(lvl)))
        return lvl.value

    def run(self, n_steps, sigma_final=None, u_recv=None):
        """March n_steps levels.  sigma_final: list of float64 CUDA tensors
        [M_i] (or None); u_recv: list of float64 CUDA tensors [n_steps][R_i]
        (or None) for the receivers' field at every level."""
        def pointers(ts, need):
            if ts is None:
                return None
            arr = (ctypes.c_void_p * self.n)()
            for i, t in enumerate(ts):
                if t is not None:
                    assert t.is_cuda and t.is_contiguous() and t.element_size() == 8 and t.numel() >= need(i)
                    arr[i] = t.data_ptr()
            return arr
        sf = pointers(sigma_final, lambda i: self.sizes[i])
        ur = pointers(u_recv, lambda i: n_steps * self.receivers[i])
        _check(self._lib.wfp_batch_run(self._h, int(n_steps), ur, sf))

    def set_levels(self, n_levels=None):
        """Per-instance level counts (each instance's own N_t; None or an
        entry <= 0: no limit)."""
        if n_levels is None:
            _check(self._lib.wfp_batch_set_levels(self._h, None))
            return
        arr = (ctypes.c_int64 * self.n)(*[int(v) for v in n_levels])
        _check(self._lib.wfp_batch_set_levels(self._h, arr))

    def reset(self):
        _check(self._lib.wfp_batch_reset(self._h))

    def autotune(self, trial_levels=5):
        """Time every launch shape from level 0 and keep the fastest; returns
        (rows_per_block, xcd_remap, spread_pass)."""
        r = ctypes.c_int32()
        x = ctypes.c_int32()
        sp = ctypes.c_int32()
        _check(self._lib.wfp_batch_autotune(self._h, int(trial_levels), ctypes.byref(r), ctypes.byref(x),
                                            ctypes.byref(sp)))
        return r.value, x.value, sp.value

    def set_shape(self, rows_per_block, xcd_remap, spread_pass):
        _check(self._lib.wfp_batch_set_shape(self._h, int(rows_per_block), int(xcd_remap), int(spread_pass)))

    def plan(self, i):
        """Instance i's plan (borrowed: valid while the batch lives)."""
        h = self._lib.wfp_batch_plan(self._h, int(i))
        if not h:
            raise WFPError(WFP_EINVAL, self._lib.wfp_last_error().decode())
        return Plan._borrow(self._lib, h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.wfp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
