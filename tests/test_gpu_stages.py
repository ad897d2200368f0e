"""Per-kernel parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes span several 64-wide tiles, and n = 48 (coarsest grid 6) gives ragged
tiles along every axis.  FP64 kernels must agree with the oracle to rounding
(FMA contraction and summation order are the only differences); FP32 kernels
to FP32 rounding of the same arithmetic."""
import numpy as np
import pytest

from paper_1611_09638_amd import inputs

pytestmark = pytest.mark.gpu

SIZES = [(32, 8), (48, 6), (64, 8)]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    return t.detach().cpu().numpy()


_PHI = {}


def evolved_phi(orc, n, coarse_n):
    """A potential from a few oracle steps on a lognormal density: strongly
    deformed (compression limiter active), positive definite."""
    key = (n, coarse_n)
    if key not in _PHI:
        box = 250.0 * n / 32
        rho = inputs.lognormal_density(n, box, 1.5, 40 + n)
        phi, _, st = orc.solve(rho, box, orc.Config(max_outer=6, coarse_n=coarse_n))
        _PHI[key] = (phi / (box / n) ** 2, orc.normalize(rho), st)
    return _PHI[key]


@pytest.mark.parametrize("n,cn", SIZES)
def test_normalize_meshmass_source_smooth(torch_cuda, orc, n, cn):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    phi, m, st = evolved_phi(orc, n, cn)
    rec = binding.Recon(n, binding.Config(coarse_n=cn))
    box = 250.0 * n / 32
    rho = inputs.lognormal_density(n, box, 1.5, 40 + n) * 3.7
    assert rel(host(rec.normalize(dev(torch, rho))), orc.normalize(rho)) < 1e-15
    M_g = host(rec.meshmass(dev(torch, phi), dev(torch, m)))
    M_o = orc.meshmass(phi, m)
    assert rel(M_g, M_o) < 1e-13
    b_g, rms_g = rec.source(dev(torch, phi), dev(torch, M_o))
    b_o = orc.source(phi, M_o)
    t_o, rb = orc.source_terms(phi, M_o)
    assert rel(host(b_g), b_o) < 1e-11
    assert abs(rms_g - np.sqrt(np.mean((rb - M_o) ** 2))) < 1e-12 * rms_g
    if n == 32:  # this potential has cells compressed past xi_m: the compression limiter is exercised
        assert st["min_lambda0"] < 0.1
    assert rel(host(rec.smooth(dev(torch, M_o))), orc.smooth(M_o)) < 1e-15
    d_g = host(rec.delta_r(dev(torch, phi)))
    assert rel(d_g, orc.delta_r(phi)) < 1e-14
    if n % 64 == 0:
        _outer_variants_agree(torch, rec, phi, m, M_o)
    else:
        with pytest.raises(binding.ReconError):
            rec.smooth(dev(torch, M_o), variant=2)


def _outer_variants_agree(torch, rec, phi, m, M):
    """The gather and LDS-streaming forms of the outer step's passes give the
    same node values bit for bit; only sums are grouped differently."""
    Ms = [rec.meshmass(dev(torch, phi), dev(torch, m), variant=v) for v in (1, 2)]
    assert torch.equal(Ms[0], Ms[1])
    src = [rec.source(dev(torch, phi), dev(torch, M), variant=v) for v in (1, 2)]
    assert rel(host(src[0][0]), host(src[1][0])) < 1e-15
    assert abs(src[0][1] - src[1][1]) <= 1e-14 * src[0][1]
    sm = [rec.smooth(dev(torch, M), variant=v) for v in (1, 2)]
    assert torch.equal(sm[0], sm[1])


@pytest.mark.parametrize("n", [128, 256])
def test_outer_passes_streamed(torch_cuda, orc, n):
    """The deformed-mesh mass, the limited source and the smoothing (App. A)
    in their LDS-streaming form (the solver's from 256^3; several tiles and
    i-chunks) against the oracle, on a strongly deformed mesh: displacements
    of up to 13 cells and cells compressed below xi_m, where the compression
    limiter acts.  Node values equal the gather kernels' bit for bit."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rng = np.random.default_rng(700 + n)
    x = np.arange(n) * (2 * np.pi / n)
    X = np.meshgrid(x, x, x, indexing="ij")
    amp = 0.93 / (2 * np.sin(3 * np.pi / n)) ** 2
    # triad entries 1 - 0.93 cos (x), at least 0.5 (y, z): positive definite,
    # with lambda_0 down to about 0.07 < xi_m
    phi = amp * (np.cos(3 * X[0]) + 0.15 * np.cos(5 * X[1] + 1.0) + 0.5 * np.cos(2 * X[2] + 2.0))
    phi += 0.002 * rng.normal(size=phi.shape)
    m = orc.normalize(inputs.lognormal_density(n, 1000.0, 1.0, 70 + n))
    rec = binding.Recon(n, binding.Config())
    M_g = host(rec.meshmass(dev(torch, phi), dev(torch, m), variant=2))
    M_o = orc.meshmass(phi, m)
    assert rel(M_g, M_o) < 1e-13
    t_o, _ = orc.source_terms(phi, M_o)
    assert (t_o > M_o.mean() - M_o + 1e-3).any()  # the compression limiter acts somewhere
    assert orc.count_not_pd(phi) == 0
    b_g, rms_g = rec.source(dev(torch, phi), dev(torch, M_o), variant=2)
    assert rel(host(b_g), orc.source(phi, M_o)) < 1e-11
    assert abs(rms_g - np.sqrt(np.mean((M_o.mean() - M_o) ** 2))) < 1e-12 * rms_g
    assert rel(host(rec.smooth(dev(torch, M_o), variant=2)), orc.smooth(M_o)) < 1e-15
    _outer_variants_agree(torch, rec, phi, m, M_o)


@pytest.mark.parametrize("n,cn", SIZES + [(128, 8), (256, 8)])
@pytest.mark.parametrize("first", [0, 1])
def test_rbgs_sweep_fp64_and_fp32(torch_cuda, orc, n, cn, first):
    """Both sweep kernels (fused two-colour where n is a multiple of 16, and
    per-colour) against the oracle; the two kernels round identically.  The
    fused kernel runs its narrow tiles with short chunks below 256 and its
    wide streaming tiles at 256 (two tiles along k in FP32)."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(coarse_n=cn))
    rng = np.random.default_rng(100 + n + first)
    a = np.exp(1.5 * rng.normal(size=(n, n, n)))
    u, b = rng.normal(size=(2, n, n, n))
    variants = (1, 2) if n % 16 == 0 else (1,)
    for scale in (1.0, 1.0 / 16):
        uo = orc.rbgs_sweep(u, a, b, scale=scale, first=first)
        ug = [host(rec.rbgs(dev(torch, u), dev(torch, a), dev(torch, b), scale=scale, first=first, variant=v))
              for v in variants]
        for x in ug:
            assert rel(x, uo) < 1e-13
            assert np.array_equal(x, ug[0])
    a32, u32, b32 = (x.astype(np.float32).astype(np.float64) for x in (a, u, b))
    if n == 48:
        # level 24 of this hierarchy is no multiple of 16
        h = n // 2
        for dt in (torch.float32, torch.float64):
            with pytest.raises(binding.ReconError):
                rec.rbgs(dev(torch, u32[:h, :h, :h], dt), dev(torch, a32[:h, :h, :h], dt),
                         dev(torch, b32[:h, :h, :h], dt), variant=2)
    uo = orc.rbgs_sweep(u32, a32, b32, first=first)
    ug = [host(rec.rbgs(dev(torch, u32, torch.float32), dev(torch, a32, torch.float32),
                        dev(torch, b32, torch.float32), first=first, variant=v)) for v in variants]
    for x in ug:
        assert rel(x, uo) < 2e-6
        assert np.array_equal(x, ug[0])


@pytest.mark.parametrize("n,cn", SIZES)
def test_residual_restrict_prolong(torch_cuda, orc, n, cn):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(coarse_n=cn))
    rng = np.random.default_rng(200 + n)
    a = np.exp(rng.normal(size=(n, n, n)))
    u, b = rng.normal(size=(2, n, n, n))
    e = rng.normal(size=(n // 2,) * 3)
    for scale in (1.0, 0.25):
        assert rel(host(rec.residual(dev(torch, u), dev(torch, a), dev(torch, b), scale)),
                   orc.residual(u, a, b, scale)) < 1e-14
        assert rel(host(rec.apply(dev(torch, u), dev(torch, a), scale)), orc.apply(u, a, scale)) < 1e-14
    assert rel(host(rec.restrict(dev(torch, u))), orc.restrict(u)) < 1e-15
    assert rel(host(rec.prolong_add(dev(torch, u), dev(torch, e))), orc.prolong_add(u, e)) < 1e-15
    f32 = lambda x: dev(torch, x, torch.float32)  # noqa: E731
    q = lambda x: x.astype(np.float32).astype(np.float64)  # noqa: E731
    assert rel(host(rec.residual(f32(u), f32(a), f32(b))), orc.residual(q(u), q(a), q(b))) < 1e-5
    assert rel(host(rec.restrict(f32(u))), orc.restrict(q(u))) < 1e-6
    assert rel(host(rec.prolong_add(f32(u), f32(e))), orc.prolong_add(q(u), q(e))) < 1e-6


@pytest.mark.parametrize("n", [64, 128, 256, 384])
def test_streaming_operator_kernels(torch_cuda, orc, n):
    """The LDS-streaming residual and Krylov direction kernels against the
    per-node gather kernels (same arithmetic, same face order) and the oracle,
    with coefficients that hit the a_min floor.  They stream 128-wide tiles,
    so an edge of 64 is rejected; at 384 there are three tiles along k."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(coarse_n=6 if n == 384 else 8))
    rng = np.random.default_rng(300 + n)
    a = np.exp(2.0 * rng.normal(size=(n, n, n)))
    a[rng.random((n, n, n)) < 0.05] = 0.0  # empty cells: floored faces
    u, b, z, p_old = rng.normal(size=(4, n, n, n))
    if n % 128:
        for dt in (torch.float64, torch.float32):
            with pytest.raises(binding.ReconError):
                rec.residual(dev(torch, u, dt), dev(torch, a, dt), dev(torch, b, dt), 1.0, variant=2)
        with pytest.raises(binding.ReconError):
            rec.direction(dev(torch, z), None, dev(torch, a), 0.5, True, variant=2)
        return
    for scale in (1.0, 0.25):
        r1 = host(rec.residual(dev(torch, u), dev(torch, a), dev(torch, b), scale, variant=1))
        r2 = host(rec.residual(dev(torch, u), dev(torch, a), dev(torch, b), scale, variant=2))
        assert np.abs(r2 - r1).max() <= 1e-15 * np.abs(r1).max()
        assert rel(r2, orc.residual(u, a, b, scale)) < 1e-14
    f32 = lambda x: dev(torch, x, torch.float32)  # noqa: E731
    q32 = lambda x: x.astype(np.float32).astype(np.float64)  # noqa: E731
    r1 = host(rec.residual(f32(u), f32(a), f32(b), 0.25, variant=1))
    assert rel(r1, orc.residual(q32(u), q32(a), q32(b), 0.25)) < 1e-5
    r2 = host(rec.residual(f32(u), f32(a), f32(b), 0.25, variant=2))
    assert np.abs(r2 - r1).max() <= 1e-6 * np.abs(r1).max()
    beta = -0.37
    for zt, zq in ((torch.float64, lambda x: x), (torch.float32, q32)):
        for first in (True, False):
            out = [rec.direction(dev(torch, z, zt), dev(torch, p_old), dev(torch, a), beta, first, variant=v)
                   for v in (1, 2)]
            (p1, qv1, pq1), (p2, qv2, pq2) = [(host(pn), host(qv), pq) for pn, qv, pq in out]
            p_ref = zq(z) if first else zq(z) + beta * p_old
            assert np.array_equal(p1, p2)
            # z + beta p is contracted to one fused multiply-add on the GPU
            assert np.abs(p2 - p_ref).max() <= 2.3e-16 * np.abs(p_ref).max()
            assert np.abs(qv2 - qv1).max() <= 1e-15 * np.abs(qv1).max()
            q_ref = orc.apply(p_ref, a)
            assert rel(qv2, q_ref) < 1e-14
            assert abs(pq2 - pq1) <= 1e-13 * abs(pq1)
            assert abs(pq2 - float(np.dot(p_ref.ravel(), q_ref.ravel()))) <= 1e-12 * abs(pq1)
    # the previous step's solution update, deferred into the direction pass:
    # same direction and product, and u + alpha p_old (one FMA) in both variants
    alpha_u = 0.8125
    u_ref = u + alpha_u * p_old
    for v in (1, 2):
        ug = dev(torch, u)
        pn, qv, pq = rec.direction(dev(torch, z), dev(torch, p_old), dev(torch, a), beta, False, variant=v, u=ug,
                                   alpha_u=alpha_u)
        p0, q0, pq0 = rec.direction(dev(torch, z), dev(torch, p_old), dev(torch, a), beta, False, variant=v)
        assert torch.equal(pn, p0) and torch.equal(qv, q0) and pq == pq0
        assert np.abs(host(ug) - u_ref).max() <= 2.3e-16 * np.abs(u_ref).max()
        if v == 1:
            u1 = host(ug)
        else:
            assert np.array_equal(host(ug), u1)
    with pytest.raises(binding.ReconError):
        ug = dev(torch, u)
        rec.direction(dev(torch, z), dev(torch, p_old), dev(torch, a), beta, True, variant=2, u=ug, alpha_u=1.0)
    # FP32 directions (the mixed solver's): p_new is z + beta p_old rounded to
    # FP32, q and p.q are the FP64 product of exactly the stored values, and the
    # deferred update adds alpha times the stored p_old
    z32, po32 = z.astype(np.float32), p_old.astype(np.float32)
    for first in (True, False):
        ug = dev(torch, u)
        pn, qv, pq = rec.direction(dev(torch, z32), None if first else dev(torch, po32), dev(torch, a), beta, first,
                                   variant=2, u=None if first else ug, alpha_u=alpha_u, p_dtype=torch.float32)
        assert pn.dtype == torch.float32
        p32 = host(pn).astype(np.float64)
        p_ref = z32.astype(np.float64) + (0.0 if first else beta * po32.astype(np.float64))
        if first:
            assert np.array_equal(p32, p_ref)
        else:  # one rounding to FP32 (the FP64 sum may be contracted to an FMA)
            assert np.abs(p32 - p_ref).max() <= 2.0 ** -24 * (1 + 1e-12) * np.abs(p_ref).max()
            u_ref = u + alpha_u * po32.astype(np.float64)
            assert np.abs(host(ug) - u_ref).max() <= 2.3e-16 * np.abs(u_ref).max()
        q_ref = orc.apply(p32, a)
        assert rel(host(qv), q_ref) < 1e-14
        assert abs(pq - float(np.dot(p32.ravel(), q_ref.ravel()))) <= 1e-12 * abs(pq)
    with pytest.raises(binding.ReconError):  # FP32 directions need an FP32 z
        rec.direction(dev(torch, z), None, dev(torch, a), beta, True, variant=2, p_dtype=torch.float32)


@pytest.mark.parametrize("n", [48, 64, 128, 256])
def test_fused_residual_restriction(torch_cuda, orc, n):
    """The V-cycle's coarse right-hand side R (b - scale A u) in one fused
    pass against the residual and restriction kernels one after the other
    (bitwise: same arithmetic, same order) and against the oracle, in FP64
    and FP32.  It needs a coarse edge that is a multiple of 32 (48 is
    rejected); at 256 the coarse grid has four tiles along k."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(coarse_n=6 if n == 48 else 8, precision=binding.MIXED))
    rng = np.random.default_rng(500 + n)
    a = np.exp(2.0 * rng.normal(size=(n, n, n)))
    a[rng.random((n, n, n)) < 0.05] = 0.0  # empty cells: floored faces
    u, b = rng.normal(size=(2, n, n, n))
    if n % 64:
        with pytest.raises(binding.ReconError):
            rec.residual_restrict(dev(torch, u), dev(torch, a), dev(torch, b), 1.0, variant=2)
        return
    for scale in (1.0, 0.25):
        c1 = host(rec.residual_restrict(dev(torch, u), dev(torch, a), dev(torch, b), scale, variant=1))
        c2 = host(rec.residual_restrict(dev(torch, u), dev(torch, a), dev(torch, b), scale, variant=2))
        assert np.array_equal(c1, c2)
        assert rel(c2, orc.restrict(orc.residual(u, a, b, scale))) < 1e-14
    f32 = lambda x: dev(torch, x, torch.float32)  # noqa: E731
    q32 = lambda x: x.astype(np.float32).astype(np.float64)  # noqa: E731
    c1 = host(rec.residual_restrict(f32(u), f32(a), f32(b), 0.25, variant=1))
    c2 = host(rec.residual_restrict(f32(u), f32(a), f32(b), 0.25, variant=2))
    assert np.array_equal(c1, c2)
    assert rel(c2, orc.restrict(orc.residual(q32(u), q32(a), q32(b), 0.25))) < 1e-5


def test_streaming_transfers(torch_cuda, orc):
    """The LDS-streaming restriction and prolongation at 256^3 against the
    per-node gather kernels (bitwise, same arithmetic and order) and against
    the oracle; smaller edges are rejected."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n = 256
    rec = binding.Recon(n, binding.Config(precision=binding.MIXED))
    rng = np.random.default_rng(401)
    f = rng.normal(size=(n, n, n))
    e = rng.normal(size=(n // 2,) * 3)
    c1 = host(rec.restrict(dev(torch, f), variant=1))
    c2 = host(rec.restrict(dev(torch, f), variant=2))
    assert np.array_equal(c1, c2)
    assert rel(c2, orc.restrict(f)) < 1e-15
    u1 = host(rec.prolong_add(dev(torch, f), dev(torch, e), variant=1))
    u2 = host(rec.prolong_add(dev(torch, f), dev(torch, e), variant=2))
    assert np.array_equal(u1, u2)
    assert rel(u2, orc.prolong_add(f, e)) < 1e-15
    f32 = lambda x: dev(torch, x, torch.float32)  # noqa: E731
    assert np.array_equal(host(rec.restrict(f32(f), variant=1)), host(rec.restrict(f32(f), variant=2)))
    assert np.array_equal(host(rec.prolong_add(f32(f), f32(e), variant=1)),
                          host(rec.prolong_add(f32(f), f32(e), variant=2)))
    h = n // 2  # a level whose edge is not a multiple of 256
    with pytest.raises(binding.ReconError):
        rec.restrict(dev(torch, f[:h, :h, :h].copy()), variant=2)
    with pytest.raises(binding.ReconError):
        rec.prolong_add(dev(torch, f[:h, :h, :h].copy()), dev(torch, e[:h // 2, :h // 2, :h // 2].copy()), variant=2)


@pytest.mark.parametrize("n,cn", SIZES)
def test_vcycle_fp64_and_fp32(torch_cuda, orc, n, cn):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rng = np.random.default_rng(300 + n)
    a = np.exp(1.5 * rng.normal(size=(n, n, n)))
    r = rng.normal(size=(n, n, n))
    r -= r.mean()
    cfg_o = orc.Config(coarse_n=cn)
    zo = orc.vcycle(a, r, cfg_o)
    rec = binding.Recon(n, binding.Config(coarse_n=cn, precision=binding.MIXED))
    assert rel(host(rec.vcycle(dev(torch, a), dev(torch, r))), zo) < 1e-12
    z32 = host(rec.vcycle(dev(torch, a, torch.float32), dev(torch, r, torch.float32)))
    assert rel(z32, zo) < 1e-4


@pytest.mark.parametrize("n,cn", SIZES)
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("solver", [0, 1])
def test_mg_solve(torch_cuda, orc, n, cn, precision, solver):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rng = np.random.default_rng(400 + n)
    a = np.exp(rng.normal(size=(n, n, n)))
    b = rng.normal(size=(n, n, n))
    b -= b.mean()
    uo, cyc_o, rel_o = orc.mg_solve(a, b, orc.Config(coarse_n=cn, tol=1e-12, solver=solver))
    rec = binding.Recon(n, binding.Config(coarse_n=cn, precision=precision, solver=solver))
    ug, cyc, relg = rec.mg_solve(dev(torch, a), dev(torch, b), tol=1e-12)
    assert relg <= 1e-12
    assert rel(host(ug), uo) < 1e-9
    assert abs(host(ug).mean()) < 1e-14 * np.abs(uo).max()
    if precision == 0:
        assert cyc == cyc_o


@pytest.mark.parametrize("n", [64, 128, 192])
def test_pd_trial_counts(torch_cuda, orc, n):
    """Failing-node counts of the step trials: the per-node gather kernel and
    the LDS-streaming kernel agree exactly (same arithmetic per node), and
    both match the oracle's count on phi + 2^-j dphi (its Hessian sums in
    another order, so a node on the boundary may differ: at most 1e-5 of n^3).
    n = 192 has 3 tiles along k; the chunking takes every plane once."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(coarse_n=6 if n == 192 else 8))
    box = 250.0 * n / 32
    g = inputs.gaussian_field(n, box, 300 + n)
    phi = 0.35 * g / np.abs(g).max()
    dphi = inputs.gaussian_field(n, box, 400 + n)
    dphi *= 6.0 / np.abs(dphi).max()
    seen = set()
    for j0 in (0, 4):
        for nt in (1, 4):
            c1 = rec.pd_count(dev(torch, phi), dev(torch, dphi), j0, nt, variant=1)
            c2 = rec.pd_count(dev(torch, phi), dev(torch, dphi), j0, nt, variant=2)
            assert c1 == c2
            for t in range(nt):
                co = orc.count_not_pd(phi + np.ldexp(1.0, -(j0 + t)) * dphi)
                assert abs(c2[t] - co) <= 1e-5 * n ** 3
                seen.add(co > 0)
    assert seen == {True, False}  # both failing and passing trials were exercised
    a_o = orc.choose_step(phi, dphi, orc.Config())[1]
    assert rec.choose_step(dev(torch, phi), dev(torch, dphi)) == a_o


def test_choose_step_and_cic(torch_cuda, orc):
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n = 32
    phi, m, st = evolved_phi(orc, n, 8)
    rec = binding.Recon(n, binding.Config())
    rng = np.random.default_rng(5)
    g = inputs.gaussian_field(n, 250.0, 77)
    for amp in (0.05, 0.5, 3.0, 40.0):
        dphi = amp * g / np.abs(g).max()
        j, a_o = orc.choose_step(phi, dphi, orc.Config())
        a_g = rec.choose_step(dev(torch, phi), dev(torch, dphi))
        assert a_g == a_o
    pos = (rng.random((5000, 3)) * 250.0).astype(np.float32)
    pos[:7] = [[0, 0, 0], [249.99998, 0, 0], [7.8125, 7.8125, 7.8125], [125, 125, 125], [0, 249.99998, 3.0],
               [1e-7, 1e-7, 1e-7], [200.5, 0.1, 249.9]]
    rho_g = host(rec.cic(dev(torch, pos), 250.0))
    rho_o = orc.cic_particles(pos, n, 250.0)
    assert np.abs(rho_g - rho_o).max() < 1e-12
    assert abs(rho_g.sum() - 5000) < 1e-9


@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("amp,s_max,axis,j_exp", [
    (20.0, 1.0, 0, 3), (20.0, 100.0, 0, 2), (20.0, 0.5, 2, 4), (0.5, 1.0, 2, 0)])
def test_choose_step_single_mode_closed_form(torch_cuda, orc, n, amp, s_max, axis, j_exp):
    """Step control against the closed form of a single Fourier mode (Sec. II):
    dphi = A sin(theta x_axis), theta = 2 pi / 16 scaled to the grid, shifts
    nodes by at most A sin(theta) and bends the triad to 1 - 4 A sin^2(theta/2)
    at worst; the step is the first 2^-j passing both bounds.  Covers a binding
    shift bound (j = 3, 4), a binding PD bound (j = 2) and a full step."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    theta = 2 * np.pi / 16
    i = np.arange(n)
    X = np.meshgrid(i, i, i, indexing="ij")
    dphi = amp * np.sin(theta * X[axis])
    phi = 0.3 / (4 * np.sin(theta / 2) ** 2) * np.cos(theta * X[(axis + 1) % 3])
    rec = binding.Recon(n, binding.Config(s_max=s_max))
    a_g = rec.choose_step(dev(torch, phi), dev(torch, dphi))
    assert a_g == 2.0 ** -j_exp
    assert orc.choose_step(phi, dphi, orc.Config(s_max=s_max)) == (j_exp, 2.0 ** -j_exp)


@pytest.mark.parametrize("n", [16, 32, 48, 64, 128, 256])
@pytest.mark.parametrize("first", [0, 1])
def test_prolongation_folded_into_the_sweep(torch_cuda, orc, n, first):
    """The V-cycle's coarse correction folded into its first post-smoothing
    sweep (App. A multigrid) on every kind of level the fused sweep runs on
    (narrow tiles with 4- and 8-plane chunks below 256, the streaming tiles at
    256; 16 takes its correction from the 8^3 coarsest level): equal bit for
    bit to the prolongation's own pass followed by the sweep, in FP64 and
    FP32, and to the oracle's prolongation and sweep in FP64."""
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    rec = binding.Recon(n, binding.Config(precision=binding.MIXED, coarse_n=6 if n == 48 else 8))
    rng = np.random.default_rng(900 + first + n)
    a = np.exp(1.5 * rng.normal(size=(n, n, n)))
    u, b = rng.normal(size=(2, n, n, n))
    e = rng.normal(size=(n // 2,) * 3)
    ug = [rec.prolong_sweep(dev(torch, u), dev(torch, e), dev(torch, a), dev(torch, b), scale=0.25, first=first,
                            variant=v) for v in (1, 2)]
    assert torch.equal(ug[0], ug[1])
    uo = orc.rbgs_sweep(orc.prolong_add(u, e), a, b, scale=0.25, first=first)
    assert rel(host(ug[1]), uo) < 1e-13
    f = lambda x: dev(torch, x, torch.float32)  # noqa: E731
    ug = [rec.prolong_sweep(f(u), f(e), f(a), f(b), scale=0.25, first=first, variant=v) for v in (1, 2)]
    assert torch.equal(ug[0], ug[1])


def test_stage_outputs_must_not_overlap_inputs(torch_cuda):
    """An output that overlaps an input (whole or in part) is rejected with
    RECON_E_ARG before anything is launched; the same calls on separate arrays
    run."""
    import ctypes
    torch = torch_cuda
    from paper_1611_09638_amd import binding
    n = 32
    rec = binding.Recon(n, binding.Config())
    L, ctx = binding.lib(), rec._ctx
    E_ARG = -1

    def P(t):
        return ctypes.c_void_p(t.data_ptr())

    f = torch.rand((n, n, n), dtype=torch.float64, device="cuda") + 0.5
    g = torch.rand((n, n, n), dtype=torch.float64, device="cuda") + 0.5
    big = torch.rand(2 * n ** 3, dtype=torch.float64, device="cuda") + 0.5
    half = big[n ** 3 // 2:]  # starts inside the first n^3 values of big
    assert L.recon_stage_apply(ctx, P(f), P(g), n, 1.0, P(f)) == E_ARG
    assert L.recon_stage_apply(ctx, P(big), P(g), n, 1.0, P(half)) == E_ARG
    assert L.recon_stage_residual(ctx, P(f), P(g), P(f), n, 1.0, P(g), 0, 0) == E_ARG
    assert L.recon_stage_delta_r(ctx, P(f), P(f)) == E_ARG
    assert L.recon_stage_meshmass(ctx, P(f), P(g), P(g), 0) == E_ARG
    assert L.recon_stage_smooth(ctx, P(half), P(big), 0) == E_ARG
    assert L.recon_stage_restrict(ctx, P(f), n, P(f), 0, 0) == E_ARG
    assert L.recon_stage_residual_restrict(ctx, P(f), P(g), P(f), n, 1.0, P(g), 0, 0) == E_ARG
    assert L.recon_stage_rbgs(ctx, P(f), P(f), P(g), n, 1.0, 0, 0, 0) == E_ARG
    assert b"overlap" in L.recon_last_error(ctx)
    assert L.recon_solve(ctx, P(g), n, 250.0, 0.0, P(f), P(f), None) == E_ARG
    out = torch.empty_like(f)
    assert L.recon_stage_apply(ctx, P(f), P(g), n, 1.0, P(out)) == 0
    assert L.recon_stage_delta_r(ctx, P(f), P(out)) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
