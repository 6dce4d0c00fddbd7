"""The Gaussian dome of Sec. 5.2 (h = hbar + A exp(-alpha (d/a)^2), no
initial wind, mean geopotential g hbar) on the HIP path:

  * the initial spectrum (grid values from the workload, transformed by the
    plan) and three MLSDC(3,2,2,1/2) steps (fine T31 with 3 Gauss-Lobatto
    nodes, coarse T15 with 2, one sweep per level, dt = 120 s) against the
    oracle at the parity tolerance, 1e-12 normwise per field;
  * the temporal order of the GPU's SDC(3,4) at T15 after 30 minutes:
    errors at dt = 450, 225, 112.5 s against SDC(5,8) at 112.5 s fall by
    2^4 per halving (observed orders within 3.5 .. 4.5), the order of
    collocation with three Gauss-Lobatto nodes after four sweeps (Sec. 4.2).
"""
import math

import pytest
import torch

import workload
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
    a = a.detach().cpu()
    b = b.detach().cpu() if torch.is_tensor(b) else torch.as_tensor(b)
    nb = torch.linalg.vector_norm(b).item()
    return torch.linalg.vector_norm(a - b).item() / (nb if nb > 0 else 1.0)


def dome_state_gpu(pk, plan, N, I):
    mu = plan.latitudes()[0]
    grid = torch.tensor(workload.dome_grid(mu, I)[None], device="cuda")
    x = torch.zeros(3, workload.nspec(N), dtype=torch.complex128, device="cuda")
    x[0] = plan.forward(grid)[0]
    return x


def test_dome_mlsdc_parity(pk):
    print("CASE dome MLSDC(3,2,2,1/2) T31/T15", flush=True)
    par = pk.swe_params(phibar=workload.dome_phibar())
    op = OW.SWEParams(phibar=workload.dome_phibar())
    pf, pc = pk.Plan(31, 48, 96), pk.Plan(15, 24, 48)
    x = dome_state_gpu(pk, pf, 31, 96)
    g = OH.Grid(31, 48, 96)
    ox = torch.zeros(3, workload.nspec(31), dtype=torch.complex128)
    ox[0] = g.sh_forward(torch.tensor(workload.dome_grid(g.mu.numpy(), 96))[None])[0]
    assert relerr(x[0], ox[0]) < TOL
    st = pk.Stepper(pk.Level(pf, par, pk.SDC_GAUSS_LOBATTO, 3), pk.Level(pc, par, pk.SDC_GAUSS_LOBATTO, 2),
                    niter=2, nsweep_fine=1, nsweep_coarse=1)
    of = OS.Level(OW.SWEProblem(31, 48, 96, op), "lobatto", 3)
    oc = OS.Level(OW.SWEProblem(15, 24, 48, op), "lobatto", 2)
    R, P = OS.spectral_transfer(31, 15)
    for k in range(3):
        x = st.step(120.0, x)
        ox = OS.mlsdc_step(of, oc, 120.0, ox, niter=2, restrict_space=R, interp_space=P)
        for f in range(3):
            assert relerr(x[f], ox[f]) < TOL, (k, f)


def test_dome_sdc_temporal_order(pk):
    print("CASE dome SDC(3,4) order T15", flush=True)
    par = pk.swe_params(phibar=workload.dome_phibar())
    plan = pk.Plan(15, 24, 48)
    x0 = dome_state_gpu(pk, plan, 15, 48)

    def run(nodes, K, dt, T=1800.0):
        st = pk.Stepper(pk.Level(plan, par, pk.SDC_GAUSS_LOBATTO, nodes), None, niter=K)
        x = x0.clone()
        for _ in range(int(round(T / dt))):
            x = st.step(dt, x)
        return x

    ref = run(5, 8, 112.5)
    err = [(run(3, 4, dt)[0] - ref[0]).abs().max().item() for dt in (450.0, 225.0, 112.5)]
    orders = [math.log2(err[i] / err[i + 1]) for i in range(2)]
    assert all(3.5 < o < 4.5 for o in orders), (err, orders)
