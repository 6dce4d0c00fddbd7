"""Hand-written adjoint: transposes of the SH pair, the tendency, the solve and
the whole MLSDC step, checked by dot-product identities, against torch
autograd through the FP64 CPU oracle (the reference gradient), against the
oracle's forward-mode directional derivatives (whole-step dot products
<J d, w> = <d, J^T w>, stored values), and against central finite differences
on the 20-step T127/T63 integration; the tendency and one step of the
T1023/T511 configuration by dot products with central differences of the
GPU's own forward maps."""
import json
import math
import os

import numpy as np
import pytest
import torch

import workload
from oracle import sdc as OS
from oracle import sht as OH
from oracle import swe as OW

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07923_amd as pk
    pk.lib()
    return pk


_G = {}


def ogrid(N, J, I):
    if (N, J, I) not in _G:
        _G[(N, J, I)] = OH.Grid(N, J, I)
    return _G[(N, J, I)]


def rdot(a, b):
    """Real inner product sum Re a Re b + Im a Im b (or sum a b for real)."""
    a, b = a.detach().cpu(), b.detach().cpu()
    if a.is_complex():
        return (a.real * b.real + a.imag * b.imag).sum().item()
    return (a * b).sum().item()


def relerr(a, b):
    a, b = a.detach().cpu(), b.detach().cpu()
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


def crandn(shape, gen):
    return torch.randn(shape, dtype=torch.float64, generator=gen) + 1j * torch.randn(shape, dtype=torch.float64,
                                                                                      generator=gen)


def seeded(N, seed, scales=(100.0, 1e-5, 1e-5)):
    raw = torch.tensor(workload.raw_spectrum(N, seed))
    return raw * torch.tensor(scales, dtype=torch.float64)[:, None]


# T511 (384 latitude pairs) takes the matrix-core analysis in the transposed synthesis
@pytest.mark.parametrize("N,J,I,F", [(31, 48, 96, 2), (40, 64, 128, 3), (511, 768, 1536, 2)])
def test_sh_pair_adjoint_dot(pk, N, J, I, F):
    print("CASE sh adjoint dot", N, J, I, F, flush=True)
    gen = torch.Generator().manual_seed(N)
    plan = pk.Plan(N, J, I)
    x = crandn((F, OH.nspec(N)), gen).cuda()
    h = torch.randn(F, J, I, dtype=torch.float64, generator=gen).cuda()
    lhs = rdot(plan.inverse(x), h)
    rhs = rdot(x, plan.inverse_adj(h))
    print("synthesis dot", N, abs(lhs - rhs) / abs(lhs), flush=True)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    s = crandn((F, OH.nspec(N)), gen).cuda()
    lhs = rdot(plan.forward(h), s)
    rhs = rdot(h, plan.forward_adj(s))
    print("analysis dot", N, abs(lhs - rhs) / abs(lhs), flush=True)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("N,J,I,S", [(31, 48, 96, 1), (63, 96, 192, 2)])
def test_tendency_adjoint_vs_autograd(pk, N, J, I, S):
    """VJP of (F_I, F_E) against torch autograd through the oracle."""
    print("CASE tendency adjoint", N, J, I, S, flush=True)
    g = ogrid(N, J, I)
    p = OW.SWEParams()
    gen = torch.Generator().manual_seed(7 + N)
    states = torch.stack([seeded(N, 90 + s) for s in range(S)])
    lfi = crandn(states.shape, gen)
    lfe = crandn(states.shape, gen)
    plan = pk.Plan(N, J, I)
    got = pk.tendency_adj(plan, pk.swe_params(), states.cuda(), lfi.cuda(), lfe.cuda())
    for s in range(S):
        x = states[s].clone().requires_grad_(True)
        fi = OW.f_implicit(x, N, p)
        fe = OW.f_explicit(x, g, p)
        loss = (fi.real * lfi[s].real + fi.imag * lfi[s].imag).sum() + \
               (fe.real * lfe[s].real + fe.imag * lfe[s].imag).sum()
        loss.backward()
        for f in range(3):
            assert relerr(got[s, f], x.grad[f]) < 1e-12, (s, f, relerr(got[s, f], x.grad[f]))


@pytest.mark.parametrize("N,J,I", [(1023, 1536, 3072), (127, 192, 384)])
def test_tendency_adjoint_dot_central_difference(pk, N, J, I):
    """<J d, w> = <d, J^T w> for the tendency on the GPU, with J d from central
    differences of the GPU tendency.  F_I is linear and F_E quadratic in the
    state (products of linear functions of it), so the central difference
    (F(x + d) - F(x - d)) / 2 is exactly J(x) d up to rounding, for a
    direction as large as the state.  At T1023 (3072-point rows) the
    transposed grid products run through the HBM workspace instead of LDS;
    T127 checks the LDS kernel the same way."""
    print("CASE tendency adjoint dot", N, flush=True)
    seed = {1023: 1004, 127: 1001}[N]
    x = torch.tensor(workload.state(N, seed), device="cuda")
    gen = torch.Generator().manual_seed(17)
    deg = torch.tensor(np.concatenate([np.arange(m, N + 1) for m in range(N + 1)]))
    m0 = torch.tensor(np.concatenate([np.full(N + 1 - m, m) for m in range(N + 1)]) == 0)
    d = crandn(x.shape, gen) * (deg + 1.0) ** -1.5
    d[:, m0] = d[:, m0].real.to(torch.complex128)
    d[:, deg == 0] = 0
    for f in range(3):                              # the size of the state, field by field
        d[f] *= torch.linalg.vector_norm(x[f].cpu()) / torch.linalg.vector_norm(d[f])
    d = d.to("cuda")
    w_fi, w_fe = crandn(x.shape, gen).to("cuda"), crandn(x.shape, gen).to("cuda")
    plan = pk.Plan(N, J, I)
    par = pk.swe_params()
    fip, fep = pk.tendency(plan, par, (x + d)[None].contiguous())
    fim, fem = pk.tendency(plan, par, (x - d)[None].contiguous())
    lhs = rdot((fip[0] - fim[0]) / 2, w_fi) + rdot((fep[0] - fem[0]) / 2, w_fe)
    lam = pk.tendency_adj(plan, par, x[None].contiguous(), w_fi[None].contiguous(), w_fe[None].contiguous())
    rhs = rdot(d, lam[0])
    scale = abs(rdot((fep[0] - fem[0]) / 2, w_fe)) + abs(rdot((fip[0] - fim[0]) / 2, w_fi))
    print("dot", lhs, rhs, abs(lhs - rhs) / scale, flush=True)
    assert abs(lhs - rhs) <= 1e-10 * scale


def test_step_adjoint_T1023_dot_central_difference(pk):
    """<J d, w> = <d, J^T w> for one step of the large configuration (T1023 /
    T511, Gauss-Radau 6 / 4 points, 2 + 2 sweeps x 4, dt = 60 s), J d from
    central differences of the GPU step with a direction of 1e-4 of the
    state: the step is a polynomial of high degree in the state, so the
    difference carries an O(eps^2) error, well under the bound."""
    print("CASE step adjoint T1023 dot", flush=True)
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(1023, 1536, 3072), par, pk.SDC_RADAU_RIGHT, 6)
    lc = pk.Level(pk.Plan(511, 768, 1536), par, pk.SDC_RADAU_RIGHT, 4)
    st = pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2)
    N = 1023
    x = torch.tensor(workload.state(N, 1004), device="cuda")
    gen = torch.Generator().manual_seed(23)
    deg = torch.tensor(np.concatenate([np.arange(m, N + 1) for m in range(N + 1)]))
    m0 = torch.tensor(np.concatenate([np.full(N + 1 - m, m) for m in range(N + 1)]) == 0)
    d = crandn(x.shape, gen) * (deg + 1.0) ** -1.5
    d[:, m0] = d[:, m0].real.to(torch.complex128)
    d[:, deg == 0] = 0
    for f in range(3):
        d[f] *= 1e-4 * torch.linalg.vector_norm(x[f].cpu()) / torch.linalg.vector_norm(d[f])
    d = d.to("cuda")
    w = crandn(x.shape, gen)
    for f in range(3):                              # weights of the size of each field's inverse
        w[f] /= torch.linalg.vector_norm(x[f].cpu())
    w = w.to("cuda")
    yp, ym = st.step(60.0, x + d), st.step(60.0, x - d)
    lhs = rdot((yp - ym) / 2, w)
    rhs = rdot(d, st.step_adj(60.0, x, w))
    print("dot", lhs, rhs, abs(lhs - rhs) / abs(lhs), flush=True)
    assert abs(lhs - rhs) <= 1e-7 * abs(lhs)


@pytest.mark.parametrize("which", ["fi", "fe"])
def test_tendency_adjoint_one_cotangent(pk, which):
    """The entry point with one of the two cotangents NULL (T31, 2 states)."""
    print("CASE tendency adjoint one cotangent", which, flush=True)
    N, J, I, S = 31, 48, 96, 2
    g = ogrid(N, J, I)
    p = OW.SWEParams()
    gen = torch.Generator().manual_seed(11)
    states = torch.stack([seeded(N, 95 + s) for s in range(S)])
    lam = crandn(states.shape, gen)
    plan = pk.Plan(N, J, I)
    if which == "fi":
        got = pk.tendency_adj(plan, pk.swe_params(), states.cuda(), lam_fi=lam.cuda())
    else:
        got = pk.tendency_adj(plan, pk.swe_params(), states.cuda(), lam_fe=lam.cuda())
    for s in range(S):
        x = states[s].clone().requires_grad_(True)
        out = OW.f_implicit(x, N, p) if which == "fi" else OW.f_explicit(x, g, p)
        (out.real * lam[s].real + out.imag * lam[s].imag).sum().backward()
        for f in range(3):
            assert relerr(got[s, f], x.grad[f]) < 1e-12, (which, s, f, relerr(got[s, f], x.grad[f]))


def test_solve_adjoint_dot(pk):
    N = 63
    gen = torch.Generator().manual_seed(3)
    plan = pk.Plan(N, 96, 192)
    par = pk.swe_params()
    b = crandn((2, 3, OH.nspec(N)), gen).cuda()
    y = crandn((2, 3, OH.nspec(N)), gen).cuda()
    for h in (0.0, 150.0, 600.0):
        lhs = rdot(pk.solve(plan, par, h, b), y)
        rhs = rdot(b, pk.solve_adj(plan, par, h, y))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _oracle_levels(specs):
    lev = []
    for (N, J, I, kind, nn) in specs:
        prob = OW.SWEProblem.__new__(OW.SWEProblem)
        prob.N, prob.grid, prob.p, prob.n_eval, prob.n_solve = N, ogrid(N, J, I), OW.SWEParams(), 0, 0
        lev.append(OS.Level(prob, kind, nn))
    return lev


CASES = [
    # (fine, coarse or None, niter, nsweep_fine, nsweep_coarse, dt)
    ((31, 48, 96, "lobatto", 3), (15, 24, 48, "lobatto", 2), 2, 2, 2, 600.0),
    ((31, 48, 96, "lobatto", 5), (15, 24, 48, "lobatto", 3), 2, 1, 1, 600.0),
    ((31, 48, 96, "radau", 4), (15, 24, 48, "radau", 3), 2, 1, 2, 600.0),
    ((31, 48, 96, "lobatto", 3), None, 3, 1, 1, 600.0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_step_adjoint_vs_autograd(pk, case):
    """lam_n = J^T lam_np1 of one MLSDC (or SDC) step against torch autograd
    through the oracle's step (the FP64 CPU reference gradient)."""
    fs, cs, niter, nsf, nsc, dt = CASES[case]
    print("CASE step adjoint", fs, cs, niter, nsf, nsc, flush=True)
    kinds = {"lobatto": pk.SDC_GAUSS_LOBATTO, "radau": pk.SDC_RADAU_RIGHT}
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(*fs[:3]), par, kinds[fs[3]], fs[4])
    lc = pk.Level(pk.Plan(*cs[:3]), par, kinds[cs[3]], cs[4]) if cs else None
    stepper = pk.Stepper(lf, lc, niter=niter, nsweep_fine=nsf, nsweep_coarse=nsc)
    gen = torch.Generator().manual_seed(11 + case)
    st = torch.tensor(workload.state(31, 1000))
    lam = crandn(st.shape, gen)
    got = stepper.step_adj(dt, st.cuda(), lam.cuda())
    levels = _oracle_levels([fs] + ([cs] if cs else []))
    x = st.clone().requires_grad_(True)
    if cs:
        R, P = OS.spectral_transfer(fs[0], cs[0])
        y = OS.mlsdc_step(levels[0], levels[1], dt, x, niter=niter, nsweep_fine=nsf, nsweep_coarse=nsc,
                          restrict_space=R, interp_space=P)
    else:
        y = OS.mlsdc_step(levels[0], None, dt, x, niter=niter, nsweep_fine=nsf)
    loss = (y.real * lam.real + y.imag * lam.imag).sum()
    loss.backward()
    for f in range(3):
        e = relerr(got[f], x.grad[f])
        print("step adjoint", case, f, e, flush=True)
        assert e < 1e-12, (f, e)


def _loss(theta):
    """L = 0.5 sum_n [|Phi'^0_n|^2 + 2 sum_{m>=1} |Phi'^m_n|^2] = (1/4 pi) int Phi'^2 (unit sphere)."""
    phi = theta[0]
    N = int((math.isqrt(8 * phi.numel() + 1) - 3) // 2)
    w = torch.where(OH.orders(N).to(phi.device) == 0, 1.0, 2.0).to(torch.float64)
    return 0.5 * (w * (phi.real ** 2 + phi.imag ** 2)).sum()


def _c3_stepper(pk):
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(127, 192, 384), par, pk.SDC_GAUSS_LOBATTO, 5)
    lc = pk.Level(pk.Plan(63, 96, 192), par, pk.SDC_GAUSS_LOBATTO, 3)
    return pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2)


def test_integrate_gradient_vs_finite_differences(pk):
    """T127/T63, GL 5/3, 2+2 sweeps x 4, dt = 300 s, 20 steps with per-step
    checkpoints; gradient of L(Phi'(T)) w.r.t. the initial vorticity against
    central differences (eps = 1e-6 relative) in 32 seeded directions."""
    print("CASE integrate FD", flush=True)
    stepper = _c3_stepper(pk)
    th0 = torch.tensor(workload.state(127, 1003)).cuda()
    dt, nsteps = 300.0, 20
    x = th0.clone().requires_grad_(True)
    L = _loss(pk.integrate(x, stepper, dt, nsteps))
    L.backward()
    grad_z = x.grad[1].clone()
    zn = torch.linalg.vector_norm(th0[1]).item()
    dirs = torch.tensor(workload.directions(127, 32, 3000, zn)).cuda()
    eps = 1e-6
    worst = 0.0
    for k in range(32):
        d = dirs[k]
        xp, xm = th0.clone(), th0.clone()
        xp[1] += eps * d
        xm[1] -= eps * d
        for _ in range(nsteps):
            xp = stepper.step(dt, xp)
            xm = stepper.step(dt, xm)
        fd = ((_loss(xp) - _loss(xm)) / (2 * eps)).item()
        an = rdot(grad_z, d)
        e = abs(fd - an) / max(abs(an), 1e-300)
        worst = max(worst, e)
    print("FD worst relative error", worst, flush=True)
    assert worst < 1e-5


def test_integrate_gradient_vs_cpu_reference(pk):
    """The same gradient against torch autograd through the oracle (one step
    at T127/T63, and three steps of the T31/T15 pair)."""
    print("CASE integrate vs CPU gradient", flush=True)
    for (fine, coarse, nsteps, dt, seed) in (((127, 192, 384), (63, 96, 192), 1, 300.0, 1003),
                                            ((31, 48, 96), (15, 24, 48), 3, 600.0, 1000)):
        par = pk.swe_params()
        lf = pk.Level(pk.Plan(*fine), par, pk.SDC_GAUSS_LOBATTO, 5)
        lc = pk.Level(pk.Plan(*coarse), par, pk.SDC_GAUSS_LOBATTO, 3)
        stepper = pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2)
        th0 = torch.tensor(workload.state(fine[0], seed))
        x = th0.clone().cuda().requires_grad_(True)
        _loss(pk.integrate(x, stepper, dt, nsteps)).backward()
        levels = _oracle_levels([fine + ("lobatto", 5), coarse + ("lobatto", 3)])
        R, P = OS.spectral_transfer(fine[0], coarse[0])
        xo = th0.clone().requires_grad_(True)
        y = xo
        for _ in range(nsteps):
            y = OS.mlsdc_step(levels[0], levels[1], dt, y, niter=4, nsweep_fine=2, nsweep_coarse=2,
                              restrict_space=R, interp_space=P)
        _loss(y).backward()
        e = relerr(x.grad[1], xo.grad[1])
        print("gradient vs CPU reference", fine, nsteps, e, flush=True)
        assert e < 1e-12


JVP_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_jvp.json")


@pytest.mark.parametrize("name", ["T31_T15_3steps", "T127_T63_1step"])
def test_integrate_gradient_vs_oracle_jvp(pk, name):
    """Whole-integration dot-product identity <J d, w> = <d, J^T w> with w =
    dL/dTheta(T): the oracle's forward-mode derivatives dL_k along the seeded
    vorticity perturbations d_k (stored; tests/golden/make_adjoint_jvp.py)
    against the GPU adjoint's gradient dotted with the same d_k."""
    print("CASE integrate vs oracle jvp", name, flush=True)
    with open(JVP_GOLDEN) as f:
        c = json.load(f)[name]
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(*c["fine"]), par, pk.SDC_GAUSS_LOBATTO, 5)
    lc = pk.Level(pk.Plan(*c["coarse"]), par, pk.SDC_GAUSS_LOBATTO, 3)
    stepper = pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2)
    N = c["fine"][0]
    th0 = torch.tensor(workload.state(N, c["seed_state"]))
    x = th0.clone().cuda().requires_grad_(True)
    _loss(pk.integrate(x, stepper, c["dt"], c["nsteps"])).backward()
    dirs = torch.tensor(workload.directions(N, c["ndirs"], c["seed_dirs"],
                                            torch.linalg.vector_norm(th0[1]).item()))
    got = np.array([rdot(x.grad[1], dirs[k]) for k in range(c["ndirs"])])
    ref = np.array(c["dL"])
    e = np.abs(got - ref).max() / np.abs(ref).max()
    print("whole-step dot identity", name, e, flush=True)
    assert e < 1e-12


def test_integrate_graph_replays_match_eager(pk):
    """The captured forward and adjoint steps give the eager results, replay
    after replay, with eager work in between."""
    print("CASE integrate graph vs eager", flush=True)
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(31, 48, 96), par, pk.SDC_GAUSS_LOBATTO, 5)
    lc = pk.Level(pk.Plan(15, 24, 48), par, pk.SDC_GAUSS_LOBATTO, 3)
    stepper = pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2)
    th0 = torch.tensor(workload.state(31, 1000)).cuda()
    results = []
    for graph in (False, True, True):
        x = th0.clone().requires_grad_(True)
        y = pk.integrate(x, stepper, 600.0, 3, graph=graph)
        _loss(y).backward()
        torch.cuda.synchronize()
        results.append((y.detach().clone(), x.grad.clone()))
        stepper.step(600.0, th0)                      # eager work between the replays
    for y, gr in results[1:]:
        assert torch.equal(y, results[0][0])
        assert torch.equal(gr, results[0][1])
