"""Python binding of libmlsdc_sh.so, the MI355X MLSDC-SH hot path.

Argument marshalling only: every step runs in the HIP library.  Tensors are
torch tensors on the current HIP device; spectral arrays are complex128
(m-major, see include/mlsdc_sh.h), grids float64.  Work is enqueued on
torch's current stream.  Importing works without a GPU; the library is
loaded on first use and a missing library raises immediately.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmlsdc_sh.so")

SHX_FP64, SHX_FP32, SHX_SPLIT_BF16_2, SHX_SPLIT_BF16_3 = 0, 1, 2, 3
SHX_TABLE_HBM, SHX_TABLE_ONTHEFLY = 0, 1
SDC_GAUSS_LOBATTO, SDC_RADAU_RIGHT = 0, 1

_lib = None


class SwePar(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("omega", ctypes.c_double), ("g", ctypes.c_double),
                ("phibar", ctypes.c_double), ("nu", ctypes.c_double)]


class MlsdcOpts(ctypes.Structure):
    _fields_ = [("niter", ctypes.c_int), ("nsweep_fine", ctypes.c_int),
                ("nsweep_coarse", ctypes.c_int), ("residual_check", ctypes.c_int)]


# name -> (restype, argtypes)
_P, _D, _I, _SZ = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
_SIGS = {
    "shx_nspec": (_SZ, [_I]),
    "shx_strerror": (ctypes.c_char_p, [_I]),
    "shx_plan_create": (_I, [_I, _I, _I, _I, _I, ctypes.POINTER(_P)]),
    "shx_plan_destroy": (None, [_P]),
    "shx_plan_latitudes": (_I, [_P, _P, _P, _P]),
    "shx_plan_legendre": (_I, [_P, _I, _I, _P]),
    "shx_plan_analysis_terms": (_I, [_P, _I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
    "shx_workspace_bytes": (_SZ, [_P, _I]),
    "sh_inverse": (_I, [_P, _I, _P, _P, _P, _SZ, _P]),
    "sh_forward": (_I, [_P, _I, _P, _P, _P, _SZ, _P]),
    "sh_legendre_synthesis": (_I, [_P, _I, _I, _P, _P, _P]),
    "sh_legendre_analysis": (_I, [_P, _I, _I, _P, _P, _P]),
    "swe_workspace_bytes": (_SZ, [_P, _I]),
    "swe_tendency": (_I, [_P, ctypes.POINTER(SwePar), _I, _P, _P, _P, _P, _SZ, _P]),
    "imex_solve": (_I, [_P, ctypes.POINTER(SwePar), _I, _D, _P, _P, _P]),
    "sdc_level_create": (_I, [_P, ctypes.POINTER(SwePar), _I, _I, ctypes.POINTER(_P)]),
    "sdc_level_destroy": (None, [_P]),
    "sdc_level_matrices": (_I, [_P, _P, _P, _P, _P]),
    "sdc_sweep_workspace_bytes": (_SZ, [_P]),
    "sdc_sweep": (_I, [_P, _D, _P, _P, _P, _P, _P, _SZ, _P]),
    "mlsdc_workspace_bytes": (_SZ, [_P, _P, ctypes.POINTER(MlsdcOpts)]),
    "mlsdc_step": (_I, [_P, _P, ctypes.POINTER(MlsdcOpts), _D, _P, _P, _P, _P, _SZ, _P]),
    "mlsdc_step_noalloc": (_I, [_P, _P, ctypes.POINTER(MlsdcOpts), _D, _P, _P, _P, _P]),
    "mlsdc_multi_workspace_bytes": (_SZ, [_P, _I]),
    "mlsdc_step_multi": (_I, [_P, _I, _I, _P, _D, _P, _P, _P, _SZ, _P]),
    "sh_inverse_adj": (_I, [_P, _I, _P, _P, _P, _SZ, _P]),
    "sh_forward_adj": (_I, [_P, _I, _P, _P, _P, _SZ, _P]),
    "swe_adj_workspace_bytes": (_SZ, [_P, _I]),
    "swe_tendency_adj": (_I, [_P, ctypes.POINTER(SwePar), _I, _P, _P, _P, _P, _P, _SZ, _P]),
    "imex_solve_adj": (_I, [_P, ctypes.POINTER(SwePar), _I, _D, _P, _P, _P]),
    "mlsdc_adj_workspace_bytes": (_SZ, [_P, _P, ctypes.POINTER(MlsdcOpts)]),
    "mlsdc_step_adj": (_I, [_P, _P, ctypes.POINTER(MlsdcOpts), _D, _P, _P, _P, _P, _SZ, _P]),
    "shx_kernel_timer_start": (_I, [_I, _I]),
    "shx_kernel_timer_stop": (_I, [_P, ctypes.POINTER(_I)]),
}
KC_LEGENDRE_SYN, KC_LEGENDRE_AN, KC_GRID, KC_SDC_NODE = 0, 1, 2, 3
EXPORTS = tuple(_SIGS)


class ShxError(RuntimeError):
    pass


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ShxError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_07923_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise ShxError(f"{what}: {lib().shx_strerror(rc).decode()} ({rc})")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, numel, name):
    import torch
    if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ShxError(f"{name}: expected a contiguous {dtype} cuda tensor with >= {numel} elements, "
                       f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return t


def nspec(N):
    return int(lib().shx_nspec(N))


class KernelTimer:
    """Times every launch of one kernel class with HIP events on its stream."""

    def __init__(self, kclass, capacity):
        self.kclass, self.capacity = kclass, capacity

    def __enter__(self):
        _check(lib().shx_kernel_timer_start(self.kclass, self.capacity), "shx_kernel_timer_start")
        self.ms = []
        return self

    def __exit__(self, *exc):
        import numpy as np
        buf = np.zeros(self.capacity, dtype=np.float32)
        n = ctypes.c_int(0)
        _check(lib().shx_kernel_timer_stop(buf.ctypes.data, ctypes.byref(n)), "shx_kernel_timer_stop")
        self.ms = buf[: n.value].astype(float).tolist()
        return False


class Workspace:
    """A reusable device byte buffer (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        return self.buf


class Plan:
    """Transform plan for truncation T_N on an nlat x nlon Gaussian grid
    (table_mode: SHX_TABLE_HBM or SHX_TABLE_ONTHEFLY)."""

    def __init__(self, N, nlat, nlon, precision=SHX_FP64, table_mode=SHX_TABLE_HBM):
        self.N, self.nlat, self.nlon, self.precision = N, nlat, nlon, precision
        self.table_mode = table_mode
        h = ctypes.c_void_p()
        _check(lib().shx_plan_create(N, nlat, nlon, precision, table_mode, ctypes.byref(h)), "shx_plan_create")
        self.h = h
        self.nspec = nspec(N)
        self.ws = Workspace()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.shx_plan_destroy(self.h)
            self.h = None

    def latitudes(self):
        import numpy as np
        mu, st, w = (np.empty(self.nlat) for _ in range(3))
        _check(lib().shx_plan_latitudes(self.h, mu.ctypes.data, st.ctypes.data, w.ctypes.data), "latitudes")
        return mu, st, w

    def legendre(self, m, n):
        import numpy as np
        out = np.empty(self.nlat // 2)
        _check(lib().shx_plan_legendre(self.h, m, n, out.ctypes.data), "shx_plan_legendre")
        return out

    def analysis_terms(self, nmax=None):
        """(table products per field, (m, latitude pair) Fourier rows read)
        of the Legendre analysis for degrees <= nmax (default N + 1), after
        the polar truncation of plans with tables."""
        t, fp = ctypes.c_longlong(), ctypes.c_longlong()
        _check(lib().shx_plan_analysis_terms(self.h, self.N + 1 if nmax is None else nmax, ctypes.byref(t),
                                             ctypes.byref(fp)), "shx_plan_analysis_terms")
        return t.value, fp.value

    def inverse(self, spec, grid=None):
        """spec complex128 [F, nspec] -> grid float64 [F, nlat, nlon]."""
        import torch
        F = spec.shape[0]
        _need(spec, torch.complex128, F * self.nspec, "spec")
        if grid is None:
            grid = torch.empty(F, self.nlat, self.nlon, dtype=torch.float64, device=spec.device)
        _need(grid, torch.float64, F * self.nlat * self.nlon, "grid")
        nb = lib().shx_workspace_bytes(self.h, F)
        ws = self.ws.get(nb)
        _check(lib().sh_inverse(self.h, F, _ptr(spec), _ptr(grid), _ptr(ws), nb, _stream()), "sh_inverse")
        return grid

    def forward(self, grid, spec=None):
        """grid float64 [F, nlat, nlon] -> spec complex128 [F, nspec]."""
        import torch
        F = grid.shape[0]
        _need(grid, torch.float64, F * self.nlat * self.nlon, "grid")
        if spec is None:
            spec = torch.empty(F, self.nspec, dtype=torch.complex128, device=grid.device)
        _need(spec, torch.complex128, F * self.nspec, "spec")
        nb = lib().shx_workspace_bytes(self.h, F)
        ws = self.ws.get(nb)
        _check(lib().sh_forward(self.h, F, _ptr(grid), _ptr(spec), _ptr(ws), nb, _stream()), "sh_forward")
        return spec

    def inverse_adj(self, grid_cot, spec_cot=None):
        """Transpose of inverse(): grid cotangent [F, nlat, nlon] -> spectral cotangent [F, nspec]."""
        import torch
        F = grid_cot.shape[0]
        _need(grid_cot, torch.float64, F * self.nlat * self.nlon, "grid_cot")
        if spec_cot is None:
            spec_cot = torch.empty(F, self.nspec, dtype=torch.complex128, device=grid_cot.device)
        _need(spec_cot, torch.complex128, F * self.nspec, "spec_cot")
        nb = lib().shx_workspace_bytes(self.h, F)
        ws = self.ws.get(nb)
        _check(lib().sh_inverse_adj(self.h, F, _ptr(grid_cot), _ptr(spec_cot), _ptr(ws), nb, _stream()),
               "sh_inverse_adj")
        return spec_cot

    def forward_adj(self, spec_cot, grid_cot=None):
        """Transpose of forward(): spectral cotangent [F, nspec] -> grid cotangent [F, nlat, nlon]."""
        import torch
        F = spec_cot.shape[0]
        _need(spec_cot, torch.complex128, F * self.nspec, "spec_cot")
        if grid_cot is None:
            grid_cot = torch.empty(F, self.nlat, self.nlon, dtype=torch.float64, device=spec_cot.device)
        _need(grid_cot, torch.float64, F * self.nlat * self.nlon, "grid_cot")
        nb = lib().shx_workspace_bytes(self.h, F)
        ws = self.ws.get(nb)
        _check(lib().sh_forward_adj(self.h, F, _ptr(spec_cot), _ptr(grid_cot), _ptr(ws), nb, _stream()),
               "sh_forward_adj")
        return grid_cot


def legendre_synthesis(plan, nfield, nmax, spec_ext, fourier_out):
    """Legendre step of the synthesis on the library layouts (see the C header)."""
    import torch
    ne = (plan.N + 1) * (plan.N + 4) // 2
    _need(spec_ext, torch.complex128, ne * nfield, "spec_ext")
    _need(fourier_out, torch.complex128, plan.nlat * (plan.N + 1) * nfield, "fourier_out")
    _check(lib().sh_legendre_synthesis(plan.h, nfield, nmax, _ptr(spec_ext), _ptr(fourier_out), _stream()),
           "sh_legendre_synthesis")
    return fourier_out


def legendre_analysis(plan, nfield, nmax, fourier_in, spec_ext):
    """Legendre step of the analysis on the library layouts (see the C header)."""
    import torch
    ne = (plan.N + 1) * (plan.N + 4) // 2
    _need(fourier_in, torch.complex128, plan.nlat * (plan.N + 1) * nfield, "fourier_in")
    _need(spec_ext, torch.complex128, ne * nfield, "spec_ext")
    _check(lib().sh_legendre_analysis(plan.h, nfield, nmax, _ptr(fourier_in), _ptr(spec_ext), _stream()),
           "sh_legendre_analysis")
    return spec_ext


def swe_params(a=6.37122e6, omega=7.292e-5, g=9.80616, phibar=2.94e4, nu=1.0e5):
    return SwePar(a, omega, g, phibar, nu)


def tendency(plan, params, state, f_impl=None, f_expl=None, ws=None):
    """state complex128 [S, 3, nspec] -> (F_I, F_E), same shape."""
    import torch
    S = state.shape[0] if state.dim() == 3 else 1
    _need(state, torch.complex128, S * 3 * plan.nspec, "state")
    if f_impl is None:
        f_impl = torch.empty_like(state)
    if f_expl is None:
        f_expl = torch.empty_like(state)
    nb = lib().swe_workspace_bytes(plan.h, S)
    w = (ws or plan.ws).get(nb)
    _check(lib().swe_tendency(plan.h, ctypes.byref(params), S, _ptr(state), _ptr(f_impl), _ptr(f_expl),
                              _ptr(w), nb, _stream()), "swe_tendency")
    return f_impl, f_expl


def tendency_adj(plan, params, state, lam_fi=None, lam_fe=None, lam_state=None, ws=None):
    """lam_state (+)= (dF_I/dTheta)^T lam_fi + (dF_E/dTheta)^T lam_fe at `state` [S, 3, nspec]."""
    import torch
    S = state.shape[0] if state.dim() == 3 else 1
    n = S * 3 * plan.nspec
    _need(state, torch.complex128, n, "state")
    for t, nm in ((lam_fi, "lam_fi"), (lam_fe, "lam_fe")):
        if t is not None:
            _need(t, torch.complex128, n, nm)
    if lam_state is None:
        lam_state = torch.zeros_like(state)
    _need(lam_state, torch.complex128, n, "lam_state")
    nb = lib().swe_adj_workspace_bytes(plan.h, S)
    w = (ws or plan.ws).get(nb)
    _check(lib().swe_tendency_adj(plan.h, ctypes.byref(params), S, _ptr(state), _ptr(lam_fi), _ptr(lam_fe),
                                  _ptr(lam_state), _ptr(w), nb, _stream()), "swe_tendency_adj")
    return lam_state


def solve_adj(plan, params, h, lam_out, lam_rhs=None):
    """Transpose of solve(): lam_rhs = (I - h F_I)^{-T} lam_out."""
    import torch
    S = lam_out.shape[0] if lam_out.dim() == 3 else 1
    _need(lam_out, torch.complex128, S * 3 * plan.nspec, "lam_out")
    if lam_rhs is None:
        lam_rhs = torch.empty_like(lam_out)
    _check(lib().imex_solve_adj(plan.h, ctypes.byref(params), S, float(h), _ptr(lam_out), _ptr(lam_rhs),
                                _stream()), "imex_solve_adj")
    return lam_rhs


def solve(plan, params, h, rhs, out=None):
    """Solve Theta - h F_I(Theta) = rhs; rhs complex128 [S, 3, nspec]."""
    import torch
    S = rhs.shape[0] if rhs.dim() == 3 else 1
    _need(rhs, torch.complex128, S * 3 * plan.nspec, "rhs")
    if out is None:
        out = torch.empty_like(rhs)
    _check(lib().imex_solve(plan.h, ctypes.byref(params), S, float(h), _ptr(rhs), _ptr(out), _stream()),
           "imex_solve")
    return out


class Level:
    """An SDC level: plan + physical constants + node set."""

    def __init__(self, plan, params, kind=SDC_GAUSS_LOBATTO, nnodes=3):
        self.plan, self.params, self.kind, self.nnodes = plan, params, kind, nnodes
        h = ctypes.c_void_p()
        _check(lib().sdc_level_create(plan.h, ctypes.byref(params), kind, nnodes, ctypes.byref(h)),
               "sdc_level_create")
        self.h = h
        self.ws = Workspace()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sdc_level_destroy(self.h)
            self.h = None

    def matrices(self):
        import numpy as np
        n = self.nnodes
        tau, Q, QE, QD = np.empty(n), np.empty((n, n)), np.empty((n, n)), np.empty((n, n))
        _check(lib().sdc_level_matrices(self.h, tau.ctypes.data, Q.ctypes.data, QE.ctypes.data,
                                        QD.ctypes.data), "sdc_level_matrices")
        return tau, Q, QE, QD

    def sweep(self, dt, theta, f_impl, f_expl, tau=None):
        """In-place sweep over node arrays complex128 [M+1, 3, nspec]."""
        import torch
        n = self.nnodes * 3 * self.plan.nspec
        for t, nm in ((theta, "theta"), (f_impl, "f_impl"), (f_expl, "f_expl")):
            _need(t, torch.complex128, n, nm)
        if tau is not None:
            _need(tau, torch.complex128, n, "tau")
        nb = lib().sdc_sweep_workspace_bytes(self.h)
        w = self.ws.get(nb)
        _check(lib().sdc_sweep(self.h, float(dt), _ptr(theta), _ptr(f_impl), _ptr(f_expl), _ptr(tau), _ptr(w),
                               nb, _stream()), "sdc_sweep")


class Stepper:
    """mlsdc_step with a persistent workspace (coarse=None: single-level SDC)."""

    def __init__(self, fine, coarse=None, niter=4, nsweep_fine=1, nsweep_coarse=1, residual_check=False):
        self.fine, self.coarse = fine, coarse
        self.opts = MlsdcOpts(niter, nsweep_fine, nsweep_coarse, int(bool(residual_check)))
        self.ws = Workspace()
        self.adj_ws = Workspace()
        self.nbytes = lib().mlsdc_workspace_bytes(fine.h, coarse.h if coarse else None, ctypes.byref(self.opts))

    def step_adj(self, dt, theta_n, lam_np1, lam_n=None):
        """Transpose of the step's Jacobian at theta_n applied to lam_np1 (recomputes the step)."""
        import torch
        n = 3 * self.fine.plan.nspec
        _need(theta_n, torch.complex128, n, "theta_n")
        _need(lam_np1, torch.complex128, n, "lam_np1")
        if lam_n is None:
            lam_n = torch.empty_like(lam_np1)
        _need(lam_n, torch.complex128, n, "lam_n")
        nb = lib().mlsdc_adj_workspace_bytes(self.fine.h, self.coarse.h if self.coarse else None,
                                             ctypes.byref(self.opts))
        w = self.adj_ws.get(nb)
        _check(lib().mlsdc_step_adj(self.fine.h, self.coarse.h if self.coarse else None, ctypes.byref(self.opts),
                                    float(dt), _ptr(theta_n), _ptr(lam_np1), _ptr(lam_n), _ptr(w), nb, _stream()),
               "mlsdc_step_adj")
        return lam_n

    def graphs(self, dt, like):
        """HIP graphs of one step and of one adjoint step at time step dt
        (captured on first use, replayed from fixed buffers): the launch
        sequence of a step is recorded once instead of being issued kernel by
        kernel from the host for every step of an integration."""
        key = float(dt)
        g = getattr(self, "_graphs", {}).get(key)
        if g is None:
            g = _StepGraphs(self, key, like)
            self._graphs = getattr(self, "_graphs", {})
            self._graphs[key] = g
        return g

    def step(self, dt, theta_n, theta_np1=None, status=None):
        import torch
        n = 3 * self.fine.plan.nspec
        _need(theta_n, torch.complex128, n, "theta_n")
        if theta_np1 is None:
            theta_np1 = torch.empty_like(theta_n)
        _need(theta_np1, torch.complex128, n, "theta_np1")
        if status is not None:
            _need(status, torch.float64, 2, "status")
        w = self.ws.get(self.nbytes)
        _check(lib().mlsdc_step(self.fine.h, self.coarse.h if self.coarse else None, ctypes.byref(self.opts),
                                float(dt), _ptr(theta_n), _ptr(theta_np1), _ptr(status), _ptr(w), self.nbytes,
                                _stream()), "mlsdc_step")
        return theta_np1

    def step_noalloc(self, dt, theta_n, theta_np1, status=None):
        """step() through mlsdc_step_noalloc: the library's per-device scratch
        array is the workspace (no device allocation by the call; the output
        tensors are the caller's)."""
        import torch
        n = 3 * self.fine.plan.nspec
        _need(theta_n, torch.complex128, n, "theta_n")
        _need(theta_np1, torch.complex128, n, "theta_np1")
        if status is not None:
            _need(status, torch.float64, 2, "status")
        _check(lib().mlsdc_step_noalloc(self.fine.h, self.coarse.h if self.coarse else None, ctypes.byref(self.opts),
                                        float(dt), _ptr(theta_n), _ptr(theta_np1), _ptr(status), _stream()),
               "mlsdc_step_noalloc")
        return theta_np1


class MultiStepper:
    """mlsdc_step_multi over levels[0] (finest) .. levels[-1] with a
    persistent workspace; nsweeps: sweeps per level and iteration (an int for
    all levels, or one per level)."""

    def __init__(self, levels, niter=4, nsweeps=1):
        self.levels = list(levels)
        L = len(self.levels)
        ns = [nsweeps] * L if isinstance(nsweeps, int) else list(nsweeps)
        if len(ns) != L:
            raise ShxError("one sweep count per level")
        self.niter = niter
        self._lv = (ctypes.c_void_p * L)(*[lv.h for lv in self.levels])
        self._ns = (ctypes.c_int * L)(*ns)
        self.ws = Workspace()
        self.nbytes = lib().mlsdc_multi_workspace_bytes(self._lv, L)
        if self.nbytes == 0:
            raise ShxError("mlsdc_step_multi: invalid level list")

    def step(self, dt, theta_n, theta_np1=None):
        import torch
        n = 3 * self.levels[0].plan.nspec
        _need(theta_n, torch.complex128, n, "theta_n")
        if theta_np1 is None:
            theta_np1 = torch.empty_like(theta_n)
        _need(theta_np1, torch.complex128, n, "theta_np1")
        w = self.ws.get(self.nbytes)
        _check(lib().mlsdc_step_multi(self._lv, len(self.levels), self.niter, self._ns, float(dt), _ptr(theta_n),
                                      _ptr(theta_np1), _ptr(w), self.nbytes, _stream()), "mlsdc_step_multi")
        return theta_np1


class _StepGraphs:
    """Captured forward and adjoint step of a Stepper (see Stepper.graphs)."""

    def __init__(self, stepper, dt, like):
        import torch
        self.x_in = like.detach().clone().contiguous()
        self.x_out = torch.empty_like(self.x_in)
        self.lam_in = torch.zeros_like(self.x_in)
        self.lam_out = torch.empty_like(self.x_in)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            # workspaces are allocated by these eager calls, before capture
            stepper.step(dt, self.x_in, self.x_out)
            stepper.step_adj(dt, self.x_in, self.lam_in, self.lam_out)
            s.synchronize()
            self.fwd = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.fwd, stream=s):
                stepper.step(dt, self.x_in, self.x_out)
            self.adj = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.adj, stream=s):
                stepper.step_adj(dt, self.x_in, self.lam_in, self.lam_out)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()

    def step(self, x):
        self.x_in.copy_(x)
        self.fwd.replay()
        return self.x_out.clone()

    def step_adj(self, x, lam):
        self.x_in.copy_(x)
        self.lam_in.copy_(lam)
        self.adj.replay()
        return self.lam_out.clone()


def _autograd():
    import torch

    class MLSDCIntegrate(torch.autograd.Function):
        """Theta(T) after `nsteps` MLSDC steps from theta0; the backward pass
        runs the hand-written adjoint step by step from per-step checkpoints."""

        @staticmethod
        def forward(ctx, theta0, stepper, dt, nsteps, graph):
            ckpt = [theta0.detach().contiguous()]
            x = ckpt[0]
            g = stepper.graphs(dt, x) if graph else None
            for _ in range(nsteps):
                x = g.step(x) if g else stepper.step(dt, x)
                ckpt.append(x)
            ctx.stepper, ctx.dt, ctx.g = stepper, dt, g
            ctx.ckpt = ckpt[:-1]
            return x.clone()

        @staticmethod
        def backward(ctx, grad_out):
            lam = grad_out.contiguous()
            for x in reversed(ctx.ckpt):
                lam = ctx.g.step_adj(x, lam) if ctx.g else ctx.stepper.step_adj(ctx.dt, x, lam)
            return lam, None, None, None, None

    class SHInverse(torch.autograd.Function):
        """sh_inverse with its transpose as the backward pass."""

        @staticmethod
        def forward(ctx, spec, plan):
            ctx.plan = plan
            return plan.inverse(spec.contiguous())

        @staticmethod
        def backward(ctx, g):
            return ctx.plan.inverse_adj(g.contiguous()), None

    class SHForward(torch.autograd.Function):
        """sh_forward with its transpose as the backward pass."""

        @staticmethod
        def forward(ctx, grid, plan):
            ctx.plan = plan
            return plan.forward(grid.contiguous())

        @staticmethod
        def backward(ctx, g):
            return ctx.plan.forward_adj(g.contiguous()), None

    return MLSDCIntegrate, SHInverse, SHForward


def integrate(theta0, stepper, dt, nsteps, graph=True):
    """Differentiable MLSDC integration (torch.autograd); with graph=True the
    forward and adjoint steps replay HIP graphs captured once per (stepper, dt)."""
    return _autograd()[0].apply(theta0, stepper, dt, nsteps, bool(graph))


def sh_inverse_fn(spec, plan):
    return _autograd()[1].apply(spec, plan)


def sh_forward_fn(grid, plan):
    return _autograd()[2].apply(grid, plan)
