"""Plans without P^m_n tables (SHX_TABLE_ONTHEFLY): every Legendre
contraction regenerates P^m_n from the restart values, and no table is
allocated.  FP64 results against the oracle at 1e-12 (normwise per field),
the exported P^m_n bit-identical to the tabulated plan's."""
import numpy as np
import pytest
import torch

import workload
from oracle import quadrature as OQ
from oracle import sdc as OS
from oracle import sht as OH
from oracle import swe as OW

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07923_amd as pk
    pk.lib()
    return pk


def relerr(a, b):
    a = a.detach().cpu() if torch.is_tensor(a) else torch.as_tensor(a)
    b = b.detach().cpu() if torch.is_tensor(b) else torch.as_tensor(b)
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


@pytest.mark.parametrize("N,J,I", [(31, 48, 96), (255, 384, 768)])
def test_onthefly_export_matches_table(pk, N, J, I):
    print("CASE onthefly export", N, flush=True)
    ph = pk.Plan(N, J, I)
    po = pk.Plan(N, J, I, table_mode=pk.SHX_TABLE_ONTHEFLY)
    omu, ost, _, _ = OQ.gauss_legendre(J)
    for m in sorted({0, 1, N // 2, N}):
        P = OH.legendre_m(m, N + 1, omu[: J // 2], ost[: J // 2])
        for n in sorted({m, m + 1, (m + N) // 2, N + 1}):
            a, b = po.legendre(m, n), ph.legendre(m, n)
            assert np.array_equal(a, b), (m, n)
            assert np.abs(a - P[n - m]).max() <= 4e-15 * max(1.0, np.abs(P[n - m]).max()), (m, n)


@pytest.mark.parametrize("N,J,I,F", [(63, 96, 192, 3), (255, 384, 768, 15), (255, 384, 768, 5)])
def test_onthefly_sh_pair(pk, N, J, I, F):
    """The transform pair of a plan without tables; 5 fields at T255 is the
    shape the tabulated plan streams its table for."""
    print("CASE onthefly sh pair", N, F, flush=True)
    g = OH.Grid(N, J, I)
    plan = pk.Plan(N, J, I, table_mode=pk.SHX_TABLE_ONTHEFLY)
    spec = torch.stack([torch.tensor(workload.raw_spectrum(N, 70 + f, 1)[0]) for f in range(F)])
    spec = spec * torch.tensor([10.0 ** (3 * (f % 4) - 6) for f in range(F)], dtype=torch.float64)[:, None]
    grid_g = plan.inverse(spec.cuda())
    grid_o = g.sh_inverse(spec)
    for f in range(F):
        assert relerr(grid_g[f], grid_o[f]) < TOL, f
    spec_g = plan.forward(grid_o.cuda())
    spec_o = g.sh_forward(grid_o)
    for f in range(F):
        assert relerr(spec_g[f], spec_o[f]) < TOL, f


def test_onthefly_tendency_and_step(pk):
    """The T127 tendency and one two-level T127/T63 (2,2) x 4 step of plans
    without tables against the oracle."""
    print("CASE onthefly tendency/step", flush=True)
    par = pk.swe_params()
    pf = pk.Plan(127, 192, 384, table_mode=pk.SHX_TABLE_ONTHEFLY)
    pc = pk.Plan(63, 96, 192, table_mode=pk.SHX_TABLE_ONTHEFLY)
    st = torch.tensor(workload.state(127, 1001))
    fi, fe = pk.tendency(pf, par, st.cuda())
    g = OH.Grid(127, 192, 384)
    p = OW.SWEParams()
    ofi, ofe = OW.f_implicit(st, 127, p), OW.f_explicit(st, g, p)
    for f in range(3):
        assert relerr(fi[f], ofi[f]) < TOL, f
        assert relerr(fe[f], ofe[f]) < TOL, f
    lf = pk.Level(pf, par, pk.SDC_GAUSS_LOBATTO, 5)
    lc = pk.Level(pc, par, pk.SDC_GAUSS_LOBATTO, 3)
    out = pk.Stepper(lf, lc, niter=4, nsweep_fine=2, nsweep_coarse=2).step(300.0, st.cuda())
    of = OS.Level(OW.SWEProblem(127, 192, 384), "lobatto", 5)
    oc = OS.Level(OW.SWEProblem(63, 96, 192), "lobatto", 3)
    R, P = OS.spectral_transfer(127, 63)
    ref = OS.mlsdc_step(of, oc, 300.0, st, niter=4, nsweep_fine=2, nsweep_coarse=2, restrict_space=R,
                        interp_space=P)
    for f in range(3):
        assert relerr(out[f], ref[f]) < TOL, f
