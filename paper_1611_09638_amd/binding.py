"""Python binding of the C ABI in ``include/recon.h`` (ctypes).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of ``librecon.so``.  PyTorch supplies device memory (the caller's
tensors and the context workspace) and the HIP stream.  There is no CPU
fallback: if the library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librecon.so")

RECON_OK = 0
ERRORS = {-1: "E_ARG", -2: "E_INPUT", -3: "E_NOT_PD", -4: "E_NO_CONVERGENCE", -5: "E_NO_TAPE", -6: "E_HIP",
          -7: "E_WORKSPACE", -8: "E_SCRATCH"}
FP64, MIXED = 0, 1
SOLVER_PCG, SOLVER_VCYCLE = 0, 1
MAX_STEPS = 64


class CConfig(ctypes.Structure):
    _fields_ = [
        ("max_outer", ctypes.c_int), ("n_pre", ctypes.c_int), ("n_post", ctypes.c_int),
        ("coarse_n", ctypes.c_int), ("coarse_sweeps", ctypes.c_int), ("max_vcycles", ctypes.c_int),
        ("max_halvings", ctypes.c_int), ("precision", ctypes.c_int), ("solver", ctypes.c_int),
        ("warm_start", ctypes.c_int), ("mass_update", ctypes.c_int), ("particle_deposit", ctypes.c_int),
        ("full_operator", ctypes.c_int),
        ("fixed_cycles", ctypes.c_int),
        ("record_tape", ctypes.c_int),
        ("tape_fp32", ctypes.c_int), ("profile", ctypes.c_int),
        ("tol", ctypes.c_double), ("outer_tol", ctypes.c_double), ("xi_m", ctypes.c_double),
        ("v_m", ctypes.c_double), ("smooth_center", ctypes.c_double), ("s_max", ctypes.c_double),
        ("a_min", ctypes.c_double),
    ]


class CStats(ctypes.Structure):
    _fields_ = [
        ("outer_steps", ctypes.c_int), ("vcycles_total", ctypes.c_int),
        ("vcycles", ctypes.c_int * MAX_STEPS),
        ("alpha", ctypes.c_double * MAX_STEPS), ("rms_sigma", ctypes.c_double * (MAX_STEPS + 1)),
        ("kappa", ctypes.c_double * (MAX_STEPS + 1)), ("rel_residual", ctypes.c_double * MAX_STEPS),
        ("min_det", ctypes.c_double), ("min_lambda0", ctypes.c_double), ("max_delta_r", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("smoother_sweeps", ctypes.c_int), ("smoother_ms", ctypes.c_double),
        ("smoother_zero_sweeps", ctypes.c_int), ("smoother_zero_ms", ctypes.c_double),
        ("alpha_limit", ctypes.c_int * MAX_STEPS),
        ("smoother_folded_sweeps", ctypes.c_int), ("smoother_folded_ms", ctypes.c_double),
    ]

    def to_dict(self):
        k = self.outer_steps
        return dict(outer_steps=k, vcycles_total=self.vcycles_total, vcycles=list(self.vcycles[:k]),
                    alpha=list(self.alpha[:k]), rms_sigma=list(self.rms_sigma[:k + 1]),
                    kappa=list(self.kappa[:k + 1]), rel_residual=list(self.rel_residual[:k]),
                    min_det=self.min_det, min_lambda0=self.min_lambda0, max_delta_r=self.max_delta_r,
                    ms_total=self.ms_total, smoother_sweeps=self.smoother_sweeps, smoother_ms=self.smoother_ms,
                    smoother_zero_sweeps=self.smoother_zero_sweeps, smoother_zero_ms=self.smoother_zero_ms,
                    alpha_limit=[("full", "shift", "pd")[x] for x in self.alpha_limit[:k]],
                    smoother_folded_sweeps=self.smoother_folded_sweeps,
                    smoother_folded_ms=self.smoother_folded_ms)


@dataclass
class Config:
    """Mirror of ``recon_config`` (defaults as ``recon_config_default``)."""
    max_outer: int = 10
    n_pre: int = 2
    n_post: int = 2
    coarse_n: int = 8
    coarse_sweeps: int = 64
    max_vcycles: int = 100
    max_halvings: int = 30
    precision: int = FP64
    solver: int = SOLVER_PCG
    warm_start: int = 1
    mass_update: int = 0
    particle_deposit: int = 0
    full_operator: int = 0
    fixed_cycles: int = 0
    record_tape: int = 0
    tape_fp32: int = 0
    profile: int = 0
    tol: float = 1e-10
    outer_tol: float = 0.0
    xi_m: float = 0.1
    v_m: float = 10.0
    smooth_center: float = 0.5
    s_max: float = 1.0
    a_min: float = 1e-3

    def c(self) -> CConfig:
        return CConfig(**{f.name: getattr(self, f.name) for f in fields(self)})


class ReconError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("recon error %d (%s): %s" % (code, ERRORS.get(code, "?"), msg))
        self.code = code


EXPORTS = {
    # name: (restype, argtypes)
}

_lib = None


def lib():
    """Load librecon.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, ll, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
    pc, ps = ctypes.POINTER(CConfig), ctypes.POINTER(CStats)
    pd, pi = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    sig = {
        "recon_config_default": (i, [pc]),
        "recon_workspace_bytes": (sz, [i, pc]),
        "recon_init": (i, [ctypes.POINTER(vp), i, pc, vp, sz, vp]),
        "recon_solve": (i, [vp, vp, i, d, d, vp, vp, ps]),
        "recon_solve_particles": (i, [vp, vp, ll, d, d, vp, vp, ps]),
        "recon_solve_noalloc": (i, [vp, i, d, d, pc, vp, vp, ps, vp]),
        "recon_backward": (i, [vp, vp, vp, vp]),
        "recon_backward_particles": (i, [vp, vp, ll, vp, vp, vp]),
        "recon_destroy": (None, [vp]),
        "recon_strerror": (ctypes.c_char_p, [i]),
        "recon_last_error": (ctypes.c_char_p, [vp]),
        "recon_stage_normalize": (i, [vp, vp, vp]),
        "recon_stage_cic": (i, [vp, vp, ll, d, vp]),
        "recon_stage_meshmass": (i, [vp, vp, vp, vp, i]),
        "recon_stage_source": (i, [vp, vp, vp, vp, pd, i]),
        "recon_stage_smooth": (i, [vp, vp, vp, i]),
        "recon_stage_apply": (i, [vp, vp, vp, i, d, vp]),
        "recon_stage_residual": (i, [vp, vp, vp, vp, i, d, vp, i, i]),
        "recon_stage_direction": (i, [vp, vp, i, vp, vp, d, i, vp, vp, pd, i, vp, d, i]),
        "recon_stage_full_residual": (i, [vp, vp, vp, vp, vp, vp, vp, pd, i]),
        "recon_stage_full_direction": (i, [vp, vp, vp, vp, i, vp, d, i, vp, vp, pd, i, vp, d, i]),
        "recon_stage_rbgs": (i, [vp, vp, vp, vp, i, d, i, i, i]),
        "recon_stage_restrict": (i, [vp, vp, i, vp, i, i]),
        "recon_stage_residual_restrict": (i, [vp, vp, vp, vp, i, d, vp, i, i]),
        "recon_stage_prolong_add": (i, [vp, vp, vp, i, i, i]),
        "recon_stage_prolong_sweep": (i, [vp, vp, vp, vp, vp, i, d, i, i, i]),
        "recon_stage_vcycle": (i, [vp, vp, vp, vp, i]),
        "recon_stage_mg_solve": (i, [vp, vp, vp, d, vp, pi, pd]),
        "recon_stage_mg_solve_full": (i, [vp, vp, vp, vp, d, vp, pi, pd]),
        "recon_stage_choose_step": (i, [vp, vp, vp, pd]),
        "recon_stage_pd_count": (i, [vp, vp, vp, i, i, i, pd, vp, vp]),
        "recon_stage_delta_r": (i, [vp, vp, vp]),
        "recon_stage_mass_change": (i, [vp, vp, vp, vp, vp]),
        "recon_stage_invert_map": (i, [vp, vp, vp, ll, d, vp, pd]),
        "recon_stage_deposit_xi": (i, [vp, vp, ll, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    EXPORTS.update(sig)
    _lib = L
    return L


def default_config() -> Config:
    c = CConfig()
    lib().recon_config_default(ctypes.byref(c))
    return Config(**{f.name: getattr(c, f.name) for f in fields(Config)})


def workspace_bytes(n: int, cfg: Config) -> int:
    c = cfg.c()
    return int(lib().recon_workspace_bytes(n, ctypes.byref(c)))


def _ptr(t: torch.Tensor | None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected dtype %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def solve_noalloc(density: torch.Tensor, box: float, cfg: Config | None = None, tol: float = 0.0,
                  phi: torch.Tensor | None = None, delta: torch.Tensor | None = None,
                  stream: torch.cuda.Stream | None = None):
    """recon_solve_noalloc: the forward solve on the library's static scratch,
    without a context or workspace.  The caller supplies the output tensors
    (phi, delta: n^3 FP64 on density's device, either may be None); the call
    itself allocates nothing.  Returns (phi, delta, stats)."""
    cfg = cfg or Config()
    n = density.shape[0]
    if density.dim() != 3 or density.shape != (n, n, n):
        raise ValueError("density must be n^3")
    st = CStats()
    c = cfg.c()
    stream = stream or torch.cuda.current_stream(density.device)
    with torch.cuda.device(density.device):
        rc = lib().recon_solve_noalloc(_ptr(density, torch.float64), n, float(box), float(tol), ctypes.byref(c),
                                       _ptr(phi, torch.float64), _ptr(delta, torch.float64), ctypes.byref(st),
                                       ctypes.c_void_p(stream.cuda_stream))
    if rc:
        raise ReconError(rc, lib().recon_strerror(rc).decode())
    return phi, delta, st.to_dict()


class Recon:
    """One library context: an n^3 grid, a config, a workspace and a stream."""

    def __init__(self, n: int, cfg: Config | None = None, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the reconstruction runs only in the HIP library")
        self.n = n
        self.cfg = cfg or Config()
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        nbytes = workspace_bytes(n, self.cfg)
        if nbytes == 0:
            raise ReconError(-1, "invalid grid size %d or config %s" % (n, self.cfg))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p()
        c = self.cfg.c()
        with torch.cuda.device(self.device):
            rc = lib().recon_init(ctypes.byref(self._ctx), n, ctypes.byref(c), _ptr(self.workspace), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream))
        if rc:
            raise ReconError(rc, lib().recon_strerror(rc).decode())
        self.last_stats = None

    def close(self):
        if self._ctx:
            lib().recon_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc:
            raise ReconError(rc, lib().recon_last_error(self._ctx).decode())

    def _field(self, dtype=torch.float64):
        return torch.empty((self.n,) * 3, dtype=dtype, device=self.device)

    # ------------------------------------------------------------- main calls
    def solve(self, density: torch.Tensor, box: float, tol: float = 0.0, want_phi=True, want_delta=True):
        phi = self._field() if want_phi else None
        delta = self._field() if want_delta else None
        st = CStats()
        self._check(lib().recon_solve(self._ctx, _ptr(density, torch.float64), self.n, float(box), float(tol),
                                      _ptr(phi), _ptr(delta), ctypes.byref(st)))
        self.last_stats = st.to_dict()
        return phi, delta, self.last_stats

    def solve_particles(self, pos: torch.Tensor, box: float, tol: float = 0.0, want_phi=True, want_delta=True):
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("positions must be [np, 3]")
        phi = self._field() if want_phi else None
        delta = self._field() if want_delta else None
        st = CStats()
        self._check(lib().recon_solve_particles(self._ctx, _ptr(pos, torch.float32), pos.shape[0], float(box),
                                                float(tol), _ptr(phi), _ptr(delta), ctypes.byref(st)))
        self.last_stats = st.to_dict()
        return phi, delta, self.last_stats

    def backward(self, grad_delta_r: torch.Tensor, grad_phi: torch.Tensor | None = None) -> torch.Tensor:
        out = self._field()
        self._check(lib().recon_backward(self._ctx, _ptr(grad_delta_r, torch.float64),
                                         _ptr(grad_phi, torch.float64), _ptr(out)))
        return out

    def backward_particles(self, pos: torch.Tensor, grad_delta_r: torch.Tensor,
                           grad_phi: torch.Tensor | None = None) -> torch.Tensor:
        """dL/d(positions) [np, 3] (FP64) of the last recorded particle-deposit
        solve; pos must be the particles of that solve."""
        out = torch.empty((pos.shape[0], 3), dtype=torch.float64, device=self.device)
        self._check(lib().recon_backward_particles(self._ctx, _ptr(pos, torch.float32), pos.shape[0],
                                                   _ptr(grad_delta_r, torch.float64), _ptr(grad_phi, torch.float64),
                                                   _ptr(out)))
        return out

    # ------------------------------------------------------------ stage calls
    def normalize(self, rho):
        m = self._field()
        self._check(lib().recon_stage_normalize(self._ctx, _ptr(rho, torch.float64), _ptr(m)))
        return m

    def cic(self, pos, box):
        rho = self._field()
        self._check(lib().recon_stage_cic(self._ctx, _ptr(pos, torch.float32), pos.shape[0], float(box), _ptr(rho)))
        return rho

    def meshmass(self, phi, m, variant=0):
        M = self._field()
        self._check(lib().recon_stage_meshmass(self._ctx, _ptr(phi, torch.float64), _ptr(m, torch.float64), _ptr(M),
                                               variant))
        return M

    def source(self, phi, M, variant=0):
        b = self._field()
        rms = ctypes.c_double()
        self._check(lib().recon_stage_source(self._ctx, _ptr(phi, torch.float64), _ptr(M, torch.float64), _ptr(b),
                                             ctypes.byref(rms), variant))
        return b, rms.value

    def smooth(self, f, variant=0):
        out = self._field()
        self._check(lib().recon_stage_smooth(self._ctx, _ptr(f, torch.float64), _ptr(out), variant))
        return out

    def apply(self, u, a, scale=1.0):
        out = torch.empty_like(u)
        self._check(lib().recon_stage_apply(self._ctx, _ptr(u, torch.float64), _ptr(a, torch.float64), u.shape[0],
                                            float(scale), _ptr(out)))
        return out

    @staticmethod
    def _dt(t):
        return 0 if t.dtype == torch.float64 else 1

    def residual(self, u, a, b, scale=1.0, variant=0):
        r = torch.empty_like(u)
        self._check(lib().recon_stage_residual(self._ctx, _ptr(u, u.dtype), _ptr(a, u.dtype), _ptr(b, u.dtype),
                                               u.shape[0], float(scale), _ptr(r), self._dt(u), variant))
        return r

    def direction(self, z, p_old, a, beta, first=False, variant=0, u=None, alpha_u=0.0, p_dtype=torch.float64):
        """(p_new, q, p_new.q): one conjugate-gradient direction and its operator
        product; with u given (FP64, updated in place) also u += alpha_u p_old.
        p_dtype: storage of p_old and p_new (float32 needs an FP32 z)."""
        p_new = self._field(p_dtype)
        q = self._field()
        pq = ctypes.c_double()
        self._check(lib().recon_stage_direction(self._ctx, _ptr(z, z.dtype), self._dt(z),
                                                None if p_old is None else _ptr(p_old, p_dtype),
                                                _ptr(a, torch.float64), float(beta), 1 if first else 0,
                                                _ptr(p_new, p_dtype), _ptr(q), ctypes.byref(pq), variant,
                                                None if u is None else _ptr(u, torch.float64), float(alpha_u),
                                                1 if p_dtype == torch.float32 else 0))
        return p_new, q, pq.value

    def full_residual(self, phi, M, u, b, variant=0, fp32_copy=False):
        """(r, r32, r.r): r = b - div(M e^-1 grad u) on the mesh of phi
        (needs full_operator=1); r32 is None unless fp32_copy."""
        r = self._field()
        r32 = self._field(torch.float32) if fp32_copy else None
        rr = ctypes.c_double()
        self._check(lib().recon_stage_full_residual(self._ctx, _ptr(phi, torch.float64), _ptr(M, torch.float64),
                                                    _ptr(u, torch.float64), _ptr(b, torch.float64), _ptr(r),
                                                    None if r32 is None else _ptr(r32, torch.float32),
                                                    ctypes.byref(rr), variant))
        return r, r32, rr.value

    def full_direction(self, phi, M, z, p_old, beta, first=False, variant=0, u=None, alpha_u=0.0,
                       p_dtype=torch.float64):
        """As direction() with the operator div(M e^-1 grad .) on the mesh of phi."""
        p_new = self._field(p_dtype)
        q = self._field()
        pq = ctypes.c_double()
        self._check(lib().recon_stage_full_direction(self._ctx, _ptr(phi, torch.float64), _ptr(M, torch.float64),
                                                     _ptr(z, z.dtype), self._dt(z),
                                                     None if p_old is None else _ptr(p_old, p_dtype),
                                                     float(beta), 1 if first else 0, _ptr(p_new, p_dtype), _ptr(q),
                                                     ctypes.byref(pq), variant,
                                                     None if u is None else _ptr(u, torch.float64), float(alpha_u),
                                                     1 if p_dtype == torch.float32 else 0))
        return p_new, q, pq.value

    def rbgs(self, u, a, b, scale=1.0, first=0, variant=0):
        u = u.clone()
        self._check(lib().recon_stage_rbgs(self._ctx, _ptr(u, u.dtype), _ptr(a, u.dtype), _ptr(b, u.dtype),
                                           u.shape[0], float(scale), first, self._dt(u), variant))
        return u

    def restrict(self, f, variant=0):
        nc = f.shape[0] // 2
        c = torch.empty((nc,) * 3, dtype=f.dtype, device=f.device)
        self._check(lib().recon_stage_restrict(self._ctx, _ptr(f, f.dtype), f.shape[0], _ptr(c), self._dt(f),
                                               variant))
        return c

    def residual_restrict(self, u, a, b, scale=1.0, variant=0):
        """c = R (b - scale A u): the V-cycle's coarse right-hand side."""
        nc = u.shape[0] // 2
        c = torch.empty((nc,) * 3, dtype=u.dtype, device=u.device)
        self._check(lib().recon_stage_residual_restrict(self._ctx, _ptr(u, u.dtype), _ptr(a, u.dtype),
                                                        _ptr(b, u.dtype), u.shape[0], float(scale), _ptr(c),
                                                        self._dt(u), variant))
        return c

    def prolong_sweep(self, u, e, a, b, scale=1.0, first=1, variant=2):
        """One fused sweep of u + P e (the V-cycle's first post-smoothing
        sweep); variant 1 prolongs in a pass of its own first."""
        u = u.clone()
        self._check(lib().recon_stage_prolong_sweep(self._ctx, _ptr(u, u.dtype), _ptr(e, u.dtype), _ptr(a, u.dtype),
                                                    _ptr(b, u.dtype), u.shape[0], float(scale), first, self._dt(u),
                                                    variant))
        return u

    def prolong_add(self, u, e, variant=0):
        u = u.clone()
        self._check(lib().recon_stage_prolong_add(self._ctx, _ptr(u, u.dtype), _ptr(e, u.dtype), u.shape[0],
                                                  self._dt(u), variant))
        return u

    def vcycle(self, a, r):
        z = torch.empty_like(r)
        self._check(lib().recon_stage_vcycle(self._ctx, _ptr(a, r.dtype), _ptr(r, r.dtype), _ptr(z), self._dt(r)))
        return z

    def mg_solve(self, a, b, tol=1e-10):
        u = self._field()
        cyc = ctypes.c_int()
        rel = ctypes.c_double()
        self._check(lib().recon_stage_mg_solve(self._ctx, _ptr(a, torch.float64), _ptr(b, torch.float64),
                                               float(tol), _ptr(u), ctypes.byref(cyc), ctypes.byref(rel)))
        return u, cyc.value, rel.value

    def mg_solve_full(self, a, phi, b, tol=1e-10):
        """div(a e^-1 grad u) = b on the mesh of phi (needs full_operator=1)."""
        u = self._field()
        cyc = ctypes.c_int()
        rel = ctypes.c_double()
        self._check(lib().recon_stage_mg_solve_full(self._ctx, _ptr(a, torch.float64), _ptr(phi, torch.float64),
                                                    _ptr(b, torch.float64), float(tol), _ptr(u),
                                                    ctypes.byref(cyc), ctypes.byref(rel)))
        return u, cyc.value, rel.value

    def choose_step(self, phi, dphi):
        alpha = ctypes.c_double()
        self._check(lib().recon_stage_choose_step(self._ctx, _ptr(phi, torch.float64), _ptr(dphi, torch.float64),
                                                  ctypes.byref(alpha)))
        return alpha.value

    def pd_count(self, phi, dphi, j0, ntrial=4, variant=0, M=None, D=None):
        counts = (ctypes.c_double * ntrial)()
        self._check(lib().recon_stage_pd_count(self._ctx, _ptr(phi, torch.float64), _ptr(dphi, torch.float64),
                                               int(j0), int(ntrial), int(variant), counts,
                                               _ptr(M, torch.float64), _ptr(D, torch.float64)))
        return [int(c) for c in counts]

    def mass_change(self, phi, M, f):
        """div(M e^-1 grad f), e = I + Hess phi: the exact mass change of a step."""
        out = self._field()
        self._check(lib().recon_stage_mass_change(self._ctx, _ptr(phi, torch.float64), _ptr(M, torch.float64),
                                                  _ptr(f, torch.float64), _ptr(out)))
        return out

    def invert_map(self, phi, pos, box, xi0=None):
        """(xi, failures): Lagrangian positions (np x 3, grid units) of float32
        particles pos on the deformed mesh of phi, by Newton from xi0 (default
        pos n / box)."""
        xi = (pos.double() * (self.n / box)).contiguous() if xi0 is None else xi0.clone()
        bad = ctypes.c_double()
        self._check(lib().recon_stage_invert_map(self._ctx, _ptr(phi, torch.float64), _ptr(pos, torch.float32),
                                                 pos.shape[0], float(box), _ptr(xi, torch.float64),
                                                 ctypes.byref(bad)))
        return xi, int(bad.value)

    def deposit_xi(self, xi):
        M = self._field()
        self._check(lib().recon_stage_deposit_xi(self._ctx, _ptr(xi, torch.float64), xi.shape[0], _ptr(M)))
        return M

    def delta_r(self, phi):
        d = self._field()
        self._check(lib().recon_stage_delta_r(self._ctx, _ptr(phi, torch.float64), _ptr(d)))
        return d


class Reconstruct(torch.autograd.Function):
    """(delta_r, phi) = Reconstruct.apply(density, recon, box); the backward
    calls the hand-written adjoint ``recon_backward``.  ``recon`` must be a
    context created with ``record_tape=1``."""

    @staticmethod
    def forward(ctx, density, recon: Recon, box: float):
        phi, delta, _ = recon.solve(density.contiguous(), box)
        ctx.recon = recon
        return delta, phi

    @staticmethod
    def backward(ctx, g_delta, g_phi):
        g_delta = torch.zeros((ctx.recon.n,) * 3, dtype=torch.float64, device=ctx.recon.device) \
            if g_delta is None else g_delta.contiguous()
        grad = ctx.recon.backward(g_delta, None if g_phi is None else g_phi.contiguous())
        return grad, None, None


class ReconstructParticles(torch.autograd.Function):
    """(delta_r, phi) = ReconstructParticles.apply(pos, recon, box) for float32
    particle positions [np, 3] deposited at their Lagrangian positions; the
    backward calls ``recon_backward_particles`` and returns dL/d(pos) in
    FP64, cast to the dtype of pos.  ``recon`` must be a context created with
    ``particle_deposit=1`` and ``record_tape=1``."""

    @staticmethod
    def forward(ctx, pos, recon: Recon, box: float):
        pos = pos.contiguous()
        phi, delta, _ = recon.solve_particles(pos, box)
        ctx.recon = recon
        ctx.save_for_backward(pos)
        return delta, phi

    @staticmethod
    def backward(ctx, g_delta, g_phi):
        (pos,) = ctx.saved_tensors
        g_delta = torch.zeros((ctx.recon.n,) * 3, dtype=torch.float64, device=ctx.recon.device) \
            if g_delta is None else g_delta.contiguous()
        grad = ctx.recon.backward_particles(pos, g_delta, None if g_phi is None else g_phi.contiguous())
        return grad.to(pos.dtype), None, None
