"""Reduced-precision Legendre contractions (FP32, split-BF16 with 2 and 3
pieces, FP32 accumulation on MFMA): error against the FP64 oracle, per field,
normwise.  Stated bounds (also in the design doc):

    mode      transform pair   tendency F_E (T127)   MLSDC step (T127/T63)
    fp32      2e-6             1e-4                  1e-6
    bf16x2    2e-5             2e-3                  5e-5
    bf16x3    2e-6             1e-4                  1e-6

The tendency bound is looser than the pair bound because F_E of vorticity
and divergence is a small difference of larger flux terms (the Coriolis
flux of the wind, the kinetic-energy Laplacian), which amplifies the relative
error of the contractions; a time step adds dt F_E to the state, so its error
is smaller again.

Each GPU error of the transform pair and of the tendency must also be within
5x of the CPU emulation's (oracle.mixed: operands rounded or split as on the
GPU, one FP32 accumulator per result), which predicts the level without
sharing the summation order.  Every test
runs on plans with tables in device memory (SHX_TABLE_HBM: the FP64 tables
rounded / split once) and on plans without tables (SHX_TABLE_ONTHEFLY: P
from the FP64 recurrence, rounded / split in registers before the product),
under the same bounds."""
import pytest
import torch

import workload
from oracle import mixed as OM
from oracle import sdc as OS
from oracle import sht as OH
from oracle import swe as OW

pytestmark = pytest.mark.gpu

MODES = {"fp32": 1, "bf16x2": 2, "bf16x3": 3}
TMODES = {"hbm": 0, "onthefly": 1}
BOUND_PAIR = {"fp32": 2e-6, "bf16x2": 2e-5, "bf16x3": 2e-6}
BOUND_TEND = {"fp32": 1e-4, "bf16x2": 2e-3, "bf16x3": 1e-4}
BOUND_STEP = {"fp32": 1e-6, "bf16x2": 5e-5, "bf16x3": 1e-6}


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


def relerr(a, b):
    a = a.detach().cpu()
    b = b.detach().cpu()
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


@pytest.mark.parametrize("tmode", list(TMODES))
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("N,J,I,F", [(31, 48, 96, 3), (40, 64, 128, 5), (255, 384, 768, 15)])
def test_pair_mixed(pk, mode, N, J, I, F, tmode):
    print("CASE mixed pair", mode, tmode, N, J, I, F, flush=True)
    g = ogrid(N, J, I)
    if N == 255:
        spec = torch.tensor(workload.states(255, workload.SEEDS["pair_T255"]).reshape(15, -1))
    else:
        spec = torch.stack([torch.tensor(workload.raw_spectrum(N, 80 + f, 1)[0]) for f in range(F)])
        spec = spec * torch.tensor([10.0 ** (3 * (f % 3) - 3) for f in range(F)], dtype=torch.float64)[:, None]
    plan = pk.Plan(N, J, I, MODES[mode], TMODES[tmode])
    grid_ref = g.sh_inverse(spec)
    spec_ref = g.sh_forward(grid_ref)
    grid_g = plan.inverse(spec.to("cuda").contiguous())
    spec_g = plan.forward(grid_ref.to("cuda").contiguous())
    key = ("pair", mode, N)
    if key not in _G:                                   # the emulation serves both table modes
        _G[key] = (OM.sh_inverse(g, spec, mode), OM.sh_forward(g, grid_ref, mode))
    grid_e, spec_e = _G[key]
    for f in range(F):
        ei, ef = relerr(grid_g[f], grid_ref[f]), relerr(spec_g[f], spec_ref[f])
        pi, pf = relerr(grid_e[f], grid_ref[f]), relerr(spec_e[f], spec_ref[f])
        assert ei < BOUND_PAIR[mode] and ef < BOUND_PAIR[mode], (f, ei, ef)
        assert ei < 5 * pi + 1e-12 and ef < 5 * pf + 1e-12, (f, ei, pi, ef, pf)


@pytest.mark.parametrize("tmode", list(TMODES))
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("nmax_plus", [0, 1])
def test_legendre_steps_mixed(pk, mode, nmax_plus, tmode):
    """The Legendre-only entry points of a reduced-precision plan, T40 on 64 x
    128 (ragged tiles), 9 fields (two MFMA column tiles), degrees <= N (some
    (m, parity) blocks then have no rows) and <= N + 1, within the pair bound
    of the FP64 oracle."""
    print("CASE mixed legendre steps", mode, nmax_plus, flush=True)
    N, J, I, F = 40, 64, 128, 9
    nmax = N + nmax_plus
    g = ogrid(N, J, I)
    plan = pk.Plan(N, J, I, MODES[mode], TMODES[tmode])
    gen = torch.Generator().manual_seed(21)
    ne = OH.nspec(N, N + 1)
    spec = torch.complex(torch.randn(ne, F, generator=gen, dtype=torch.float64),
                         torch.randn(ne, F, generator=gen, dtype=torch.float64))
    m0 = torch.tensor([m == 0 for m in OH.orders(N, N + 1).tolist()])
    spec[m0] = spec[m0].real.to(torch.complex128)
    keep = (OH.degrees(N, N + 1) <= nmax)[:, None]
    spec = torch.where(keep, spec, torch.zeros_like(spec))
    four = torch.empty(2, J // 2, N + 1, F, dtype=torch.complex128, device="cuda")
    pk.legendre_synthesis(plan, F, nmax, spec.to("cuda").contiguous(), four)
    four = four.cpu()
    got = torch.cat([four[0] + four[1], (four[0] - four[1]).flip(0)], dim=0)      # [J][N+1][F]
    for f in range(F):
        ref = g.legendre_synthesis(spec[:, f], N + 1)
        assert relerr(got[:, :, f], ref) < BOUND_PAIR[mode], ("synthesis", f)
    fin = torch.complex(torch.randn(J, N + 1, F, generator=gen, dtype=torch.float64),
                        torch.randn(J, N + 1, F, generator=gen, dtype=torch.float64))
    out = torch.zeros(ne, F, dtype=torch.complex128, device="cuda")
    pk.legendre_analysis(plan, F, nmax, fin.to("cuda").contiguous(), out)
    out = out.cpu()
    for f in range(F):
        ref = g.legendre_analysis(fin[:, :, f], torch.ones(J, dtype=torch.float64), N + 1)
        assert relerr(out[:, f][keep[:, 0]], ref[keep[:, 0]]) < BOUND_PAIR[mode], ("analysis", f)


@pytest.mark.parametrize("tmode", list(TMODES))
@pytest.mark.parametrize("mode", list(MODES))
def test_plan_tables_mixed(pk, mode, tmode):
    N, J, I = 63, 96, 192
    plan = pk.Plan(N, J, I, MODES[mode], TMODES[tmode])
    mu, st, _, _ = __import__("oracle.quadrature", fromlist=["x"]).gauss_legendre(J)
    tol = {"fp32": 1e-7, "bf16x2": 2e-5, "bf16x3": 1e-7}[mode]
    for m in (0, 5, 40, 63):
        P = OH.legendre_m(m, N + 1, mu[: J // 2], st[: J // 2])
        for n in (m, m + 1, N, N + 1):
            got = plan.legendre(m, n)
            assert abs(got - P[n - m]).max() <= tol * max(1.0, abs(P[n - m]).max()), (m, n)


@pytest.mark.parametrize("tmode", list(TMODES))
@pytest.mark.parametrize("mode", list(MODES))
def test_tendency_mixed(pk, mode, tmode):
    print("CASE mixed tendency", mode, tmode, flush=True)
    N, J, I = 127, 192, 384
    g = ogrid(N, J, I)
    st = torch.tensor(workload.state(127, 1001))
    plan = pk.Plan(N, J, I, MODES[mode], TMODES[tmode])
    fi, fe = pk.tendency(plan, pk.swe_params(), st[None].to("cuda").contiguous())
    ofe = OW.f_explicit(st, g, OW.SWEParams())
    key = ("tendency", mode)
    if key not in _G:
        _G[key] = OW.f_explicit(st, OM.MixedGrid(g, mode), OW.SWEParams())
    efe = _G[key]
    for f in range(3):
        e, pe = relerr(fe[0, f], ofe[f]), relerr(efe[f], ofe[f])
        print("tendency", mode, f, e, "emulated", pe, flush=True)
        assert e < BOUND_TEND[mode], (f, e)
        assert e < 5 * pe, (f, e, pe)


@pytest.mark.parametrize("tmode", list(TMODES))
@pytest.mark.parametrize("mode", list(MODES))
def test_mlsdc_step_mixed(pk, mode, tmode):
    """One T127/T63 step (GL 5/3, 2+2 sweeps x 4) with mixed tables on both
    levels; the error vs the FP64 oracle stays at the contraction level."""
    print("CASE mixed mlsdc", mode, tmode, flush=True)
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(127, 192, 384, MODES[mode], TMODES[tmode]), par, pk.SDC_GAUSS_LOBATTO, 5)
    lc = pk.Level(pk.Plan(63, 96, 192, MODES[mode], TMODES[tmode]), par, pk.SDC_GAUSS_LOBATTO, 3)
    st = torch.tensor(workload.state(127, 1001))
    out = pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2).step(300.0, st.to("cuda"))
    of = OS.Level(OW.SWEProblem.__new__(OW.SWEProblem), "lobatto", 5)
    of.problem.N, of.problem.grid, of.problem.p = 127, ogrid(127, 192, 384), OW.SWEParams()
    oc = OS.Level(OW.SWEProblem.__new__(OW.SWEProblem), "lobatto", 3)
    oc.problem.N, oc.problem.grid, oc.problem.p = 63, ogrid(63, 96, 192), OW.SWEParams()
    for lv in (of, oc):
        lv.problem.n_eval = lv.problem.n_solve = 0
    R, P = OS.spectral_transfer(127, 63)
    ref = OS.mlsdc_step(of, oc, 300.0, st, niter=4, nsweep_fine=2, nsweep_coarse=2, restrict_space=R,
                        interp_space=P)
    for f in range(3):
        e = relerr(out[f], ref[f])
        print("mlsdc", mode, tmode, f, e, flush=True)
        assert e < BOUND_STEP[mode], (f, e)
