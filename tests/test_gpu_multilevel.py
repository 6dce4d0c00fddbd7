"""Multi-level MLSDC (mlsdc_step_multi, the V-cycle of which Algorithm 1 is
the two-level case) on the HIP path:

  * one and two levels reproduce single-level SDC and mlsdc_step bit for
    bit (the same launches);
  * three levels (T31 / T15 / T7 with 5 / 3 / 2 Gauss-Lobatto nodes, one
    sweep per level, dt = 300 s) and four levels (T31 / T15 / T10 / T7,
    1 / 2 / 1 / 2 sweeps) against the oracle's V-cycle at the parity
    tolerance, 1e-12 normwise per field;
  * iterated to convergence, the three-level step reaches the fine
    collocation solution (the same as single-level SDC iterated to
    convergence, within 1e-11), which needs the restricted middle-level FAS
    term in the coarsest tau;
  * invalid level lists are rejected.
"""
import pytest
import torch

import workload
from oracle import sdc as OS
from oracle import swe as OW

pytestmark = pytest.mark.gpu

TOL = 1e-12
GRIDS = {31: (48, 96), 15: (24, 48), 10: (16, 32), 7: (12, 48), 63: (96, 192)}


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


def seeded(N, seed):
    raw = torch.tensor(workload.raw_spectrum(N, seed, 3))
    return raw * torch.tensor([100.0, 1e-5, 1e-5], dtype=torch.float64)[:, None]


def levels(pk, spec):
    par = pk.swe_params()
    return [pk.Level(pk.Plan(N, *GRIDS[N]), par, pk.SDC_GAUSS_LOBATTO, nodes) for N, nodes in spec]


def test_multi_one_and_two_levels_are_sdc_and_mlsdc_step(pk):
    print("CASE multi 1 and 2 levels T63/T31", flush=True)
    x = seeded(63, 91).to("cuda")
    lf, lc = levels(pk, [(63, 5), (31, 3)])
    a = pk.MultiStepper([lf, lc], niter=2, nsweeps=[2, 1]).step(300.0, x)
    b = pk.Stepper(lf, lc, niter=2, nsweep_fine=2, nsweep_coarse=1).step(300.0, x)
    assert torch.equal(a, b)
    a1 = pk.MultiStepper([lf], niter=3).step(300.0, x)
    b1 = pk.Stepper(lf, None, niter=3).step(300.0, x)
    assert torch.equal(a1, b1)


def test_multi_three_levels_parity(pk):
    print("CASE multi 3 levels T31/T15/T7", flush=True)
    spec = [(31, 5), (15, 3), (7, 2)]
    st = pk.MultiStepper(levels(pk, spec), niter=3, nsweeps=1)
    x = seeded(31, 92)
    got = st.step(300.0, x.to("cuda"))
    olv = [OS.Level(OW.SWEProblem(N, *GRIDS[N]), "lobatto", nodes) for N, nodes in spec]
    tr = [OS.spectral_transfer(31, 15), OS.spectral_transfer(15, 7)]
    ref = OS.mlsdc_step_multi(olv, 300.0, x, 3, [1, 1, 1], tr)
    for f in range(3):
        assert relerr(got[f], ref[f]) < TOL, f


def test_multi_four_levels_parity(pk):
    """The deepest V-cycle the entry point takes: T31 / T15 / T10 / T7 with
    5 / 3 / 3 / 2 nodes and 1 / 2 / 1 / 2 sweeps per level, two iterations."""
    print("CASE multi 4 levels T31/T15/T10/T7", flush=True)
    spec = [(31, 5), (15, 3), (10, 3), (7, 2)]
    ns = [1, 2, 1, 2]
    st = pk.MultiStepper(levels(pk, spec), niter=2, nsweeps=ns)
    x = seeded(31, 95)
    got = st.step(300.0, x.to("cuda"))
    olv = [OS.Level(OW.SWEProblem(N, *GRIDS[N]), "lobatto", nodes) for N, nodes in spec]
    tr = [OS.spectral_transfer(31, 15), OS.spectral_transfer(15, 10), OS.spectral_transfer(10, 7)]
    ref = OS.mlsdc_step_multi(olv, 300.0, x, 2, ns, tr)
    for f in range(3):
        assert relerr(got[f], ref[f]) < TOL, f


def test_multi_three_levels_fixed_point(pk):
    print("CASE multi 3 levels fixed point", flush=True)
    lv = levels(pk, [(31, 5), (15, 3), (7, 2)])
    x = seeded(31, 93).to("cuda")
    ml = pk.MultiStepper(lv, niter=14, nsweeps=1).step(300.0, x)
    sdc = pk.Stepper(lv[0], None, niter=40).step(300.0, x)
    for f in range(3):
        assert relerr(ml[f], sdc[f]) < 1e-11, f


def test_multi_rejects_invalid_levels(pk):
    print("CASE multi invalid levels", flush=True)
    lf, lc = levels(pk, [(31, 3), (15, 3)])
    with pytest.raises(pk.ShxError):
        pk.MultiStepper([lc, lf])                       # coarse before fine
    lr = pk.Level(pk.Plan(15, 24, 48), pk.swe_params(), pk.SDC_RADAU_RIGHT, 3)
    with pytest.raises(pk.ShxError):
        pk.MultiStepper([lf, lr])                       # mixed node kinds
    st = pk.MultiStepper([lf, lc], niter=1, nsweeps=[1, 0])
    with pytest.raises(pk.ShxError, match="invalid"):
        st.step(300.0, seeded(31, 94).to("cuda"))
