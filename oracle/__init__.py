"""FP64 CPU oracle for the nonlinear reconstruction (arXiv:1611.09638).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke()``
and by the benchmark's ``cpu_baseline`` leg.  The product path (the HIP library
and its Python binding) never imports or calls anything here, and this package
imports nothing from the product package.

Thin numpy wrappers over ``librecon_oracle.so`` (plain C, ``recon_oracle.c``:
the forward method and its reverse mode).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["recon_oracle.c"]
_LIB_PATH = os.path.join(_HERE, "librecon_oracle.so")

ORC_E = {0: "ok", -1: "E_ARG", -2: "E_INPUT", -3: "E_NOT_PD", -4: "E_NO_CONVERGENCE", -5: "E_NO_TAPE", -7: "E_NOMEM"}

MAX_STEPS = 256


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """Compile a copy of the oracle with AddressSanitizer and UBSan (any error
    aborts) into ``path``.  Loaded instead of the normal build when the
    environment variable RECON_ORACLE_LIB names it; the process must preload
    the ASan runtime."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", path] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    return path


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("max_outer", ctypes.c_int), ("n_pre", ctypes.c_int), ("n_post", ctypes.c_int),
        ("coarse_n", ctypes.c_int), ("coarse_sweeps", ctypes.c_int), ("max_vcycles", ctypes.c_int),
        ("max_halvings", ctypes.c_int), ("record_tape", ctypes.c_int), ("solver", ctypes.c_int), ("warm_start", ctypes.c_int),
        ("mass_update", ctypes.c_int), ("particle_deposit", ctypes.c_int), ("full_operator", ctypes.c_int),
        ("tol", ctypes.c_double), ("outer_tol", ctypes.c_double), ("xi_m", ctypes.c_double),
        ("v_m", ctypes.c_double), ("smooth_center", ctypes.c_double), ("s_max", ctypes.c_double),
        ("a_min", ctypes.c_double),
    ]


class OrcStats(ctypes.Structure):
    _fields_ = [
        ("outer_steps", ctypes.c_int), ("vcycles_total", ctypes.c_int),
        ("vcycles", ctypes.c_int * MAX_STEPS),
        ("alpha", ctypes.c_double * MAX_STEPS), ("rms_sigma", ctypes.c_double * MAX_STEPS),
        ("kappa", ctypes.c_double * MAX_STEPS), ("rel_residual", ctypes.c_double * MAX_STEPS),
        ("min_det", ctypes.c_double), ("min_lambda0", ctypes.c_double), ("max_delta_r", ctypes.c_double),
    ]

    def to_dict(self):
        k = self.outer_steps
        return dict(outer_steps=k, vcycles_total=self.vcycles_total,
                    vcycles=list(self.vcycles[:k]), alpha=list(self.alpha[:k]),
                    rms_sigma=list(self.rms_sigma[:k + 1]), kappa=list(self.kappa[:k + 1]),
                    rel_residual=list(self.rel_residual[:k]), min_det=self.min_det,
                    min_lambda0=self.min_lambda0, max_delta_r=self.max_delta_r)


@dataclass
class Config:
    """Solver knobs (defaults: xi_m = 1/10 and v_m = 10 from App. A/B; the rest
    are the readings of the multigrid and step control)."""
    max_outer: int = 10
    n_pre: int = 2
    n_post: int = 2
    coarse_n: int = 8
    coarse_sweeps: int = 64
    max_vcycles: int = 100
    max_halvings: int = 30
    record_tape: int = 0
    solver: int = 0  # 0: V-cycle-preconditioned CG, 1: plain V-cycle iteration
    warm_start: int = 1  # start each linear solve from the previous outer step's solution
    mass_update: int = 0  # 1: carry M by the exact mass change of App. A instead of re-gathering it
    particle_deposit: int = 0  # particle input, 1: deposit at the Lagrangian positions every step
    full_operator: int = 0  # 1: solve with div(M e^-1 grad .) instead of the x ~ xi operator
    tol: float = 1e-10
    outer_tol: float = 0.0
    xi_m: float = 0.1
    v_m: float = 10.0
    smooth_center: float = 0.5
    s_max: float = 1.0
    a_min: float = 1e-3

    def c(self) -> OrcConfig:
        return OrcConfig(**{f.name: getattr(self, f.name) for f in fields(self)})


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error %d (%s)" % (code, ORC_E.get(code, "?")))
        self.code = code


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("RECON_ORACLE_LIB", _LIB_PATH)
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        d, i, dbl, ll = _dp, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        fp = ctypes.POINTER(ctypes.c_float)
        sig = {
            "orc_cic_particles": (i, [fp, ll, i, dbl, d]),
            "orc_normalize": (i, [d, i, d]),
            "orc_meshmass": (None, [d, d, i, d]),
            "orc_smooth": (None, [d, i, dbl, d]),
            "orc_source_terms": (dbl, [d, d, i, dbl, dbl, d]),
            "orc_source": (None, [d, d, i, dbl, dbl, dbl, d]),
            "orc_apply": (None, [d, d, i, dbl, dbl, d]),
            "orc_residual": (None, [d, d, d, i, dbl, dbl, d]),
            "orc_rbgs_sweep": (None, [d, d, d, i, dbl, dbl, i]),
            "orc_rbgs_half": (None, [d, d, d, i, dbl, dbl, i]),
            "orc_vcycle": (i, [d, d, i, ctypes.POINTER(OrcConfig), d]),
            "orc_restrict": (None, [d, i, d]),
            "orc_prolong_add": (None, [d, d, i]),
            "orc_num_levels": (i, [i, i]),
            "orc_mg_solve": (i, [d, d, i, ctypes.POINTER(OrcConfig), d, d]),
            "orc_mg_solve_full": (i, [d, d, d, i, ctypes.POINTER(OrcConfig), d, d, d]),
            "orc_is_pd": (i, [d, i]),
            "orc_count_not_pd": (ctypes.c_long, [d, i]),
            "orc_max_shift": (dbl, [d, i]),
            "orc_choose_step": (i, [d, d, i, ctypes.POINTER(OrcConfig), d]),
            "orc_choose_step_mass": (i, [d, d, d, d, i, ctypes.POINTER(OrcConfig), d]),
            "orc_full_operator": (None, [d, d, d, i, d]),
            "orc_full_operator_floor": (None, [d, d, d, i, dbl, d]),
            "orc_invert_map": (i, [d, i, d, ctypes.c_long, d, i, dbl]),
            "orc_deposit_xi": (None, [d, ctypes.c_long, i, d]),
            "orc_solve_particles": (i, [fp, ll, i, dbl, ctypes.POINTER(OrcConfig), d, d, ctypes.POINTER(OrcStats)]),
            "orc_delta_r": (None, [d, i, d]),
            "orc_solve": (i, [d, i, dbl, ctypes.POINTER(OrcConfig), d, d, ctypes.POINTER(OrcStats)]),
            "orc_lambda_min": (dbl, [d]),
            "orc_det3": (dbl, [d]),
            "orc_triad_at": (None, [d, i, i, i, i, d]),
            "orc_tape_steps": (i, []),
            "orc_backward": (i, [d, d, dbl, ctypes.POINTER(OrcConfig), d]),
            "orc_backward_particles": (i, [d, d, dbl, ctypes.POINTER(OrcConfig), d]),
            "orc_full_operator_at": (None, [d, d, d, i, ctypes.POINTER(ctypes.c_long), ctypes.c_long, dbl, d]),
            "orc_tape_particles": (ctypes.c_long, []),
            "orc_eig_min_vec": (None, [d, d, d]),
            "orc_tape_clear": (None, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def cic_particles(pos: np.ndarray, n: int, box: float) -> np.ndarray:
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    rho = np.empty((n, n, n))
    rc = lib().orc_cic_particles(pos.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), pos.shape[0], n, box, _p(rho))
    if rc:
        raise OracleError(rc)
    return rho


def normalize(rho) -> np.ndarray:
    rho = _f64(rho)
    m = np.empty_like(rho)
    rc = lib().orc_normalize(_p(rho), rho.shape[0], _p(m))
    if rc:
        raise OracleError(rc)
    return m


def meshmass(phi, m) -> np.ndarray:
    phi, m = _f64(phi), _f64(m)
    M = np.empty_like(m)
    lib().orc_meshmass(_p(phi), _p(m), m.shape[0], _p(M))
    return M


def smooth(f, c0: float = 0.5) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_smooth(_p(f), f.shape[0], c0, _p(out))
    return out


def source_terms(phi, M, xi_m=0.1, v_m=10.0):
    phi, M = _f64(phi), _f64(M)
    t = np.empty_like(M)
    rb = lib().orc_source_terms(_p(phi), _p(M), M.shape[0], xi_m, v_m, _p(t))
    return t, rb


def source(phi, M, xi_m=0.1, v_m=10.0, c0=0.5) -> np.ndarray:
    phi, M = _f64(phi), _f64(M)
    b = np.empty_like(M)
    lib().orc_source(_p(phi), _p(M), M.shape[0], xi_m, v_m, c0, _p(b))
    return b


def apply(u, a, scale=1.0, a_min=1e-3) -> np.ndarray:
    u, a = _f64(u), _f64(a)
    out = np.empty_like(u)
    lib().orc_apply(_p(u), _p(a), u.shape[0], scale, a_min, _p(out))
    return out


def residual(u, a, b, scale=1.0, a_min=1e-3) -> np.ndarray:
    u, a, b = _f64(u), _f64(a), _f64(b)
    r = np.empty_like(u)
    lib().orc_residual(_p(u), _p(a), _p(b), u.shape[0], scale, a_min, _p(r))
    return r


def rbgs_sweep(u, a, b, scale=1.0, a_min=1e-3, first=0) -> np.ndarray:
    u = _f64(u).copy()
    a, b = _f64(a), _f64(b)
    lib().orc_rbgs_sweep(_p(u), _p(a), _p(b), u.shape[0], scale, a_min, first)
    return u


def rbgs_half(u, a, b, colour, scale=1.0, a_min=1e-3) -> np.ndarray:
    u = _f64(u).copy()
    a, b = _f64(a), _f64(b)
    lib().orc_rbgs_half(_p(u), _p(a), _p(b), u.shape[0], scale, a_min, colour)
    return u


def vcycle(a, r, cfg: Config | None = None) -> np.ndarray:
    cfg = cfg or Config()
    a, r = _f64(a), _f64(r)
    z = np.empty_like(r)
    c = cfg.c()
    rc = lib().orc_vcycle(_p(a), _p(r), r.shape[0], ctypes.byref(c), _p(z))
    if rc:
        raise OracleError(rc)
    return z


def restrict(f) -> np.ndarray:
    f = _f64(f)
    n = f.shape[0]
    c = np.empty((n // 2,) * 3)
    lib().orc_restrict(_p(f), n, _p(c))
    return c


def prolong_add(u, e) -> np.ndarray:
    u = _f64(u).copy()
    e = _f64(e)
    lib().orc_prolong_add(_p(u), _p(e), u.shape[0])
    return u


def mg_solve_full(a, phi, b, cfg: Config | None = None, u0=None):
    """(u, cycles, rel): div(a e^-1 grad u) = b on the mesh of phi, preconditioned
    by the x ~ xi V-cycle of a."""
    cfg = cfg or Config()
    a, phi, b = _f64(a), _f64(phi), _f64(b)
    u = np.empty_like(b)
    rel = ctypes.c_double()
    c = cfg.c()
    rc = lib().orc_mg_solve_full(_p(a), _p(phi), _p(b), a.shape[0], ctypes.byref(c),
                                 None if u0 is None else _p(_f64(u0)), _p(u), ctypes.byref(rel))
    if rc < 0:
        raise OracleError(rc)
    return u, rc, rel.value


def mg_solve(a, b, cfg: Config | None = None):
    cfg = cfg or Config()
    a, b = _f64(a), _f64(b)
    u = np.empty_like(b)
    rel = ctypes.c_double(0.0)
    c = cfg.c()
    rc = lib().orc_mg_solve(_p(a), _p(b), b.shape[0], ctypes.byref(c), _p(u), ctypes.byref(rel))
    if rc < 0:
        raise OracleError(rc)
    return u, rc, rel.value


def is_pd(phi) -> bool:
    phi = _f64(phi)
    return bool(lib().orc_is_pd(_p(phi), phi.shape[0]))


def count_not_pd(phi) -> int:
    """Nodes where I + Hess(phi) fails Sylvester's criterion."""
    phi = _f64(phi)
    return int(lib().orc_count_not_pd(_p(phi), phi.shape[0]))


def max_shift(f) -> float:
    f = _f64(f)
    return lib().orc_max_shift(_p(f), f.shape[0])


def choose_step(phi, dphi, cfg: Config | None = None, M=None, D=None):
    """(j, alpha) of the step control; with M and D also M + alpha D > 0."""
    cfg = cfg or Config()
    phi, dphi = _f64(phi), _f64(dphi)
    alpha = ctypes.c_double(0.0)
    c = cfg.c()
    if M is None:
        j = lib().orc_choose_step(_p(phi), _p(dphi), phi.shape[0], ctypes.byref(c), ctypes.byref(alpha))
    else:
        M, D = _f64(M), _f64(D)
        j = lib().orc_choose_step_mass(_p(phi), _p(dphi), _p(M), _p(D), phi.shape[0], ctypes.byref(c),
                                       ctypes.byref(alpha))
    return j, (alpha.value if j >= 0 else None)


def full_operator(phi, M, f, a_min: float = 0.0) -> np.ndarray:
    """div(M e^-1 grad f) with e = I + Hess phi: the exact mass change of App. A
    (a_min = 0), or the exact-Jacobian solve's operator, whose diagonal face
    coefficients are floored at a_min (a_min > 0)."""
    phi, M, f = _f64(phi), _f64(M), _f64(f)
    out = np.empty_like(f)
    if a_min > 0.0:
        lib().orc_full_operator_floor(_p(phi), _p(M), _p(f), phi.shape[0], float(a_min), _p(out))
    else:
        lib().orc_full_operator(_p(phi), _p(M), _p(f), phi.shape[0], _p(out))
    return out


def delta_r(phi) -> np.ndarray:
    phi = _f64(phi)
    d = np.empty_like(phi)
    lib().orc_delta_r(_p(phi), phi.shape[0], _p(d))
    return d


def lambda_min(e) -> float:
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(9)
    return lib().orc_lambda_min(_p(e))


def full_operator_at(phi, M, f, idx, a_min: float = 0.0) -> np.ndarray:
    """full_operator(phi, M, f, a_min).ravel()[idx], formed at the listed nodes only."""
    phi, M, f = _f64(phi), _f64(M), _f64(f)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx))
    lib().orc_full_operator_at(_p(phi), _p(M), _p(f), phi.shape[0],
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(idx), float(a_min), _p(out))
    return out


def triad_at(phi, i, j, k) -> np.ndarray:
    phi = _f64(phi)
    e = np.empty(9)
    lib().orc_triad_at(_p(phi), phi.shape[0], i, j, k, _p(e))
    return e.reshape(3, 3)


def det3(e) -> float:
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(9)
    return lib().orc_det3(_p(e))


def num_levels(n: int, coarse_n: int = 8) -> int:
    return lib().orc_num_levels(n, coarse_n)


def eig_min_vec(e):
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(9)
    lam = ctypes.c_double()
    v = np.empty(3)
    lib().orc_eig_min_vec(_p(e), ctypes.byref(lam), _p(v))
    return lam.value, v


def backward(grad_delta, grad_phi, box: float, cfg: Config | None = None) -> np.ndarray:
    """dL/d(density) for the last solve run with record_tape=1."""
    cfg = cfg or Config()
    gd = _f64(grad_delta)
    gp = None if grad_phi is None else _f64(grad_phi)
    out = np.empty_like(gd)
    c = cfg.c()
    rc = lib().orc_backward(_p(gd), None if gp is None else _p(gp), box, ctypes.byref(c), _p(out))
    if rc:
        raise OracleError(rc)
    return out


def backward_particles(grad_delta, grad_phi, box: float, cfg: Config | None = None) -> np.ndarray:
    """dL/d(positions) [np, 3] for the last solve_particles run with
    particle_deposit=1 and record_tape=1 (the adjoint through the inversion
    of the map and the xi-space deposit)."""
    cfg = cfg or Config()
    gd = _f64(grad_delta)
    gp = None if grad_phi is None else _f64(grad_phi)
    npart = lib().orc_tape_particles()
    if npart <= 0:
        raise OracleError(-5)
    out = np.empty((npart, 3))
    c = cfg.c()
    rc = lib().orc_backward_particles(_p(gd), None if gp is None else _p(gp), box, ctypes.byref(c), _p(out))
    if rc:
        raise OracleError(rc)
    return out


def invert_map(phi, y, xi0=None, max_iter: int = 100, tol: float = 1e-12):
    """Lagrangian positions xi (np x 3, grid units) with x(xi) = y for the
    continuous map x = xi + trilinear(D_c phi); Newton from xi0 (default y)."""
    phi = _f64(phi)
    y = _f64(y)
    xi = (y if xi0 is None else _f64(xi0)).copy()
    rc = lib().orc_invert_map(_p(phi), phi.shape[0], _p(y), y.shape[0], _p(xi), max_iter, tol)
    if rc:
        raise OracleError(rc)
    return xi


def deposit_xi(xi, n: int) -> np.ndarray:
    """CIC deposit of the particles at Lagrangian positions xi, n^3/np each."""
    xi = _f64(xi)
    M = np.empty((n, n, n))
    lib().orc_deposit_xi(_p(xi), xi.shape[0], n, _p(M))
    return M


def solve_particles(pos, n: int, box: float, cfg: Config | None = None, raise_on_error: bool = True):
    """Forward reconstruction from float32 particle positions [np, 3] in [0, box)."""
    cfg = cfg or Config()
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    phi = np.empty((n, n, n))
    dr = np.empty((n, n, n))
    st = OrcStats()
    c = cfg.c()
    rc = lib().orc_solve_particles(pos.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), pos.shape[0], n, box,
                                   ctypes.byref(c), _p(phi), _p(dr), ctypes.byref(st))
    if rc and raise_on_error:
        raise OracleError(rc)
    out = st.to_dict()
    out["status"] = rc
    return phi, dr, out


def solve(rho, box: float, cfg: Config | None = None, raise_on_error: bool = True):
    """Full forward reconstruction.  Returns (phi [length^2], delta_r, stats dict)."""
    cfg = cfg or Config()
    rho = _f64(rho)
    n = rho.shape[0]
    phi = np.empty_like(rho)
    dr = np.empty_like(rho)
    st = OrcStats()
    c = cfg.c()
    rc = lib().orc_solve(_p(rho), n, box, ctypes.byref(c), _p(phi), _p(dr), ctypes.byref(st))
    if rc and raise_on_error:
        raise OracleError(rc)
    out = st.to_dict()
    out["status"] = rc
    return phi, dr, out
