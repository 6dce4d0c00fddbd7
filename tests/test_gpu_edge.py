"""Edge and degenerate cases of the HIP path against the FP64 oracle, same
tolerance as the other parity tests (1e-12 normwise per field):

  * the smallest plans: T1 on a single latitude pair (2 x 16, one 64-lane
    tile with one active lane, one radix-8 FFT stage), T7 on the smallest
    3 * 2^k longitude count (12 x 48), T10 on 16 x 32;
  * two-node (trapezoidal) Gauss-Lobatto SDC, the smallest node set;
  * a coarse level with as many nodes as the fine one (coarsening in space
    only: the time transfers are identities), and one with the fine level's
    truncation (coarsening in time only: the spectral transfers are
    identities), through mlsdc_step and the multi-level entry point;
  * zero iterations (the step returns the spread initial value);
  * empty inputs (no fields, no states) rejected with SHX_EINVAL before any
    launch, and the adjoints' refusal of reduced-precision plans."""
import ctypes

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
    nb = torch.linalg.vector_norm(b).item()
    return torch.linalg.vector_norm(a - b).item() / (nb if nb > 0 else 1.0)


def seeded(N, seed):
    raw = torch.tensor(workload.raw_spectrum(N, seed, 3))
    return raw * torch.tensor([100.0, 1e-5, 1e-5], dtype=torch.float64)[:, None]


def oracle_problem(N, J, I):
    prob = OW.SWEProblem.__new__(OW.SWEProblem)
    prob.N, prob.grid, prob.p, prob.n_eval, prob.n_solve = N, OH.Grid(N, J, I), OW.SWEParams(), 0, 0
    return prob


@pytest.mark.parametrize("N,J,I", [(1, 2, 16), (7, 12, 48), (10, 16, 32)])
def test_smallest_plans(pk, N, J, I):
    """Transform pair (3 fields) and tendency (2 states) on the smallest
    grids the library accepts; all three are alias free."""
    print("CASE smallest plan", N, J, I, flush=True)
    g = OH.Grid(N, J, I)
    p = OW.SWEParams()
    plan = pk.Plan(N, J, I)
    mu, _, w = plan.latitudes()
    omu, _, _, ow = OQ.gauss_legendre(J)
    assert np.all(np.abs(mu - omu) <= np.spacing(np.abs(omu)) + 1e-300)
    assert np.all(np.abs(w - ow) <= np.spacing(ow))
    spec = seeded(N, 80)
    grid_g = plan.inverse(spec.to("cuda"))
    grid_o = g.sh_inverse(spec)
    for f in range(3):
        assert relerr(grid_g[f], grid_o[f]) < TOL, ("inverse", f)
    spec_g = plan.forward(grid_o.to("cuda").contiguous())
    spec_o = g.sh_forward(grid_o)
    for f in range(3):
        assert relerr(spec_g[f], spec_o[f]) < TOL, ("forward", f)
    states = torch.stack([seeded(N, 81), seeded(N, 82)])
    fi, fe = pk.tendency(plan, pk.swe_params(), states.to("cuda").contiguous())
    for s in range(2):
        ofi = OW.f_implicit(states[s], N, p)
        ofe = OW.f_explicit(states[s], g, p)
        for f in range(3):
            assert relerr(fi[s, f], ofi[f]) < TOL, ("f_implicit", s, f)
            assert relerr(fe[s, f], ofe[f]) < TOL, ("f_explicit", s, f)


def test_two_node_sdc(pk):
    """SDC with the two Gauss-Lobatto nodes (the trapezoidal rule), T31,
    three iterations, dt = 600 s."""
    print("CASE two-node SDC", flush=True)
    N, J, I = 31, 48, 96
    st = torch.tensor(workload.state(N, 1000))
    lev = pk.Level(pk.Plan(N, J, I), pk.swe_params(), pk.SDC_GAUSS_LOBATTO, 2)
    out = pk.Stepper(lev, None, niter=3).step(600.0, st.to("cuda"))
    olev = OS.Level(oracle_problem(N, J, I), "lobatto", 2)
    ref = OS.mlsdc_step(olev, None, 600.0, st, niter=3)
    for f in range(3):
        assert relerr(out[f], ref[f]) < TOL, f


def test_consecutive_sweeps_two_nodes(pk):
    """Several sweeps in a row on two-node levels: the first of two
    consecutive sweeps leaves the F of its last node to the next sweep's
    first update, which with two nodes reads and rewrites the same node
    (Theta^M = Theta^1).  Single-level SDC with 3 sweeps per iteration, and
    two levels (3 / 2 nodes) with 2 + 2 sweeps, against the oracle."""
    print("CASE consecutive sweeps, two nodes", flush=True)
    N, J, I = 31, 48, 96
    par = pk.swe_params()
    st = torch.tensor(workload.state(N, 1000))
    lev2 = pk.Level(pk.Plan(N, J, I), par, pk.SDC_GAUSS_LOBATTO, 2)
    out = pk.Stepper(lev2, None, niter=2, nsweep_fine=3).step(600.0, st.to("cuda"))
    olev2 = OS.Level(oracle_problem(N, J, I), "lobatto", 2)
    ref = OS.mlsdc_step(olev2, None, 600.0, st, niter=2, nsweep_fine=3)
    for f in range(3):
        assert relerr(out[f], ref[f]) < TOL, ("sdc", f)
    lf = pk.Level(pk.Plan(N, J, I), par, pk.SDC_GAUSS_LOBATTO, 3)
    lc = pk.Level(pk.Plan(15, 24, 48), par, pk.SDC_GAUSS_LOBATTO, 2)
    out = pk.Stepper(lf, lc, niter=2, nsweep_fine=2, nsweep_coarse=2).step(600.0, st.to("cuda"))
    of = OS.Level(oracle_problem(N, J, I), "lobatto", 3)
    oc = OS.Level(oracle_problem(15, 24, 48), "lobatto", 2)
    R, P = OS.spectral_transfer(N, 15)
    ref = OS.mlsdc_step(of, oc, 600.0, st, niter=2, nsweep_fine=2, nsweep_coarse=2, restrict_space=R,
                        interp_space=P)
    for f in range(3):
        assert relerr(out[f], ref[f]) < TOL, ("mlsdc", f)


def test_mlsdc_equal_node_counts(pk):
    """Two levels with three Gauss-Lobatto nodes each (T31 / T15): only the
    space is coarsened, the time restriction and interpolation are the
    identity."""
    print("CASE mlsdc equal nodes", flush=True)
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(31, 48, 96), par, pk.SDC_GAUSS_LOBATTO, 3)
    lc = pk.Level(pk.Plan(15, 24, 48), par, pk.SDC_GAUSS_LOBATTO, 3)
    st = torch.tensor(workload.state(31, 1000))
    out = pk.Stepper(lf, lc, niter=2, nsweep_fine=1, nsweep_coarse=1).step(600.0, st.to("cuda"))
    of = OS.Level(oracle_problem(31, 48, 96), "lobatto", 3)
    oc = OS.Level(oracle_problem(15, 24, 48), "lobatto", 3)
    R, P = OS.spectral_transfer(31, 15)
    ref = OS.mlsdc_step(of, oc, 600.0, st, niter=2, restrict_space=R, interp_space=P)
    for f in range(3):
        assert relerr(out[f], ref[f]) < TOL, f


def test_mlsdc_equal_truncation(pk):
    """Two T31 levels with three and two Gauss-Lobatto nodes: only the time
    is coarsened, restriction and interpolation in space are the identity."""
    print("CASE mlsdc equal truncation", flush=True)
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(31, 48, 96), par, pk.SDC_GAUSS_LOBATTO, 3)
    lc = pk.Level(pk.Plan(31, 48, 96), par, pk.SDC_GAUSS_LOBATTO, 2)
    st = torch.tensor(workload.state(31, 1000))
    out = pk.Stepper(lf, lc, niter=2, nsweep_fine=1, nsweep_coarse=1).step(600.0, st.to("cuda"))
    multi = pk.MultiStepper([lf, lc], niter=2, nsweeps=1).step(600.0, st.to("cuda"))
    assert torch.equal(out, multi)
    of = OS.Level(oracle_problem(31, 48, 96), "lobatto", 3)
    oc = OS.Level(oracle_problem(31, 48, 96), "lobatto", 2)
    R, P = OS.spectral_transfer(31, 31)
    ref = OS.mlsdc_step(of, oc, 600.0, st, niter=2, restrict_space=R, interp_space=P)
    for f in range(3):
        assert relerr(out[f], ref[f]) < TOL, f


def test_zero_iterations(pk):
    """niter = 0: no sweep runs and the step returns the spread initial
    value, for one and for two levels."""
    print("CASE zero iterations", flush=True)
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(31, 48, 96), par, pk.SDC_GAUSS_LOBATTO, 3)
    lc = pk.Level(pk.Plan(15, 24, 48), par, pk.SDC_GAUSS_LOBATTO, 2)
    st = torch.tensor(workload.state(31, 1000)).to("cuda")
    for coarse in (None, lc):
        out = pk.Stepper(lf, coarse, niter=0).step(600.0, st)
        assert torch.equal(out, st)


def test_empty_inputs_rejected(pk):
    """No fields / no states: SHX_EINVAL (-1) from the entry points."""
    print("CASE empty inputs", flush=True)
    L = pk.lib()
    plan = pk.Plan(31, 48, 96)
    buf = torch.zeros(4096, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    nb = L.shx_workspace_bytes(plan.h, 1)
    ws = torch.zeros(max(1, nb // 8 + 1), dtype=torch.float64, device="cuda")
    assert L.sh_inverse(plan.h, 0, p, p, ws.data_ptr(), nb, None) == -1
    assert L.sh_forward(plan.h, 0, p, p, ws.data_ptr(), nb, None) == -1
    par = pk.swe_params()
    assert L.swe_tendency(plan.h, ctypes.byref(par), 0, p, p, p, ws.data_ptr(), nb, None) == -1
    assert L.imex_solve(plan.h, ctypes.byref(par), 0, ctypes.c_double(1.0), p, p, None) == -1
    torch.cuda.synchronize()


def test_adjoint_rejects_reduced_precision(pk):
    """The adjoints are FP64 only: a plan of reduced working precision gives
    SHX_EUNSUPPORTED (and no launch)."""
    print("CASE adjoint reduced precision", flush=True)
    plan = pk.Plan(31, 48, 96, pk.SHX_FP32)
    st = seeded(31, 90)[None].to("cuda").contiguous()
    with pytest.raises(pk.ShxError, match="unsupported"):
        pk.tendency_adj(plan, pk.swe_params(), st, lam_fe=torch.ones_like(st))
    with pytest.raises(pk.ShxError, match="unsupported"):
        plan.inverse_adj(torch.zeros(1, 48, 96, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
