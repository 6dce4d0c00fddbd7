"""The large two-level configuration: fine T1023 on the 3072 x 1536 Gaussian
grid with 5 Gauss-Radau-right collocation points, coarse T511 on 1536 x 768
with 3, 2 + 2 sweeps x 4 iterations, dt = 60 s, FP64 and the reduced
precisions.

The FP64 oracle needs minutes at this size, so its results were computed once
by tests/golden/make_large_T1023.py (oracle only) and stored as the full
2-norm of every field plus the values at 512 seeded positions per field.
Each GPU result is checked
  * normwise, with the error norm estimated from the samples
    (sqrt(n / n_samples * sum |d_i|^2) / ||ref||), against 1e-12 in FP64;
    for the tendency, against the oracle's own sensitivity where that is
    larger: at T1023 the Laplacian's n(n+1) ~ 1e6 lifts the rounding noise
    of the kinetic-energy analysis at high degrees, so the oracle's
    divergence tendency moves by 5e-12 .. 4e-11 when only the rounding of
    its sums or of its Legendre functions changes
    (tests/golden/make_large_sensitivity_T1023.py: latitude order,
    synthesis degree order, complex FFTs, functions moved within their last
    bit, all of these at once, and the functions from the FP64 three-term
    recurrence as an on-the-fly transform generates them); the bound is
    1.25 times the largest of these per field.  The step is checked against
    ten times its latitude-order sensitivity (below 1e-12 here);
  * by its own full 2-norm against the stored one (a check over every entry);
and by properties that hold at any size (round trip of the pair, mass
conservation of the step)."""
import json
import math
import os

import numpy as np
import pytest
import torch

import workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "large_T1023.json")
SENS = os.path.join(HERE, "golden", "large_T1023_sensitivity.json")
TOL = 1e-12
MIXED = os.path.join(HERE, "golden", "large_T1023_mixed.json")
# Reduced precisions: the tendency's error against the FP64 oracle is bounded
# by five times the error that the CPU emulation of the same contractions
# (oracle.mixed, stored by tests/golden/make_large_mixed_T1023.py) makes on
# the full T1023 tendency, per field.  The divergence tendency is the worst
# conditioned result: the Laplacian's n(n+1) ~ 1e6 multiplies the
# contraction error of the kinetic-energy analysis at high degrees, where the
# tendency itself is small.  A 60 s step adds dt F to the state and stays
# near the contraction level.
BOUND_STEP = {1: 5e-6, 2: 3e-4, 3: 5e-6}
MODE_NAMES = {1: "fp32", 2: "bf16x2", 3: "bf16x3"}


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07923_amd as pk
    pk.lib()
    return pk


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def state(gold):
    return torch.tensor(workload.state(1023, gold["config"]["seed"]), device="cuda")


def sampled_error(x, rec):
    """(estimated normwise relative error, relative difference of the full norms)."""
    x = x.reshape(-1).detach()
    idx = torch.tensor(rec["idx"], device=x.device)
    got = x[idx].cpu()
    if "val" in rec:
        ref = torch.tensor(rec["val"], dtype=torch.float64)
    else:
        ref = torch.complex(torch.tensor(rec["re"], dtype=torch.float64), torch.tensor(rec["im"], dtype=torch.float64))
    d2 = (got - ref).abs().pow(2).sum().item()
    est = math.sqrt(d2 * x.numel() / len(rec["idx"])) / rec["norm"]
    full = abs(torch.linalg.vector_norm(x).item() - rec["norm"]) / rec["norm"]
    return est, full


def tendency_sensitivity(gold):
    """Per field, the largest stored change of the oracle's F_E under a change
    of rounding only."""
    with open(SENS) as fh:
        sens = json.load(fh)
    rows = [gold["f_explicit_order_sensitivity"]] + [v for k, v in sens.items() if k != "config"]
    return [max(r[f] for r in rows) for f in range(3)]


def check(x, recs, tol, what, sens=None, factor=10.0):
    for f, rec in enumerate(recs):
        t = max(tol, factor * sens[f]) if sens else tol
        est, full = sampled_error(x[f], rec)
        print(what, f, est, full, "bound", t, flush=True)
        assert est < t and full < t, (what, f, est, full, t)


def levels(pk, prec, tmode=0):
    par = pk.swe_params()
    lf = pk.Level(pk.Plan(1023, 1536, 3072, prec, tmode), par, pk.SDC_RADAU_RIGHT, 6)
    lc = pk.Level(pk.Plan(511, 768, 1536, prec, tmode), par, pk.SDC_RADAU_RIGHT, 4)
    return lf, lc


def test_large_tables(pk):
    """The plan's P^m_n at T1023 (double-double recurrence on the device)
    against the oracle's (long-double recurrence), at the plan's latitudes."""
    from oracle import sht as OH
    print("CASE large tables T1023", flush=True)
    plan = pk.Plan(1023, 1536, 3072)
    mu, st, _ = plan.latitudes()
    for m in (0, 1, 200, 511, 900, 1023):
        P = OH.legendre_m(m, 1024, mu[:768], st[:768])
        for n in sorted(n for n in {m, m + 1, (m + 1023) // 2, 1022, 1023, 1024} if n >= m):
            got = plan.legendre(m, n)
            ref = P[n - m]
            scale = max(1.0, np.abs(P).max())
            assert np.abs(got - ref).max() <= 4e-15 * scale, (m, n, np.abs(got - ref).max())


def test_large_pair_fp64(pk, gold, state):
    print("CASE large pair T1023 fp64", flush=True)
    plan = pk.Plan(1023, 1536, 3072)
    grid = plan.inverse(state)
    check(grid, gold["synthesis"], TOL, "synthesis")
    check(plan.forward(grid * grid), gold["analysis_of_square"], TOL, "analysis of square")
    back = plan.forward(grid)
    for f in range(3):
        e = (torch.linalg.vector_norm(back[f] - state[f]) / torch.linalg.vector_norm(state[f])).item()
        assert e < TOL, ("round trip", f, e)


def test_large_tendency_fp64(pk, gold, state):
    print("CASE large tendency T1023 fp64", flush=True)
    plan = pk.Plan(1023, 1536, 3072)
    _, fe = pk.tendency(plan, pk.swe_params(), state[None].contiguous())
    check(fe[0], gold["f_explicit"], TOL, "f_explicit", tendency_sensitivity(gold), 1.25)


def test_large_step_fp64(pk, gold, state):
    """One T1023/T511 Radau 5/3 step against the oracle; Phi'^0_0 (the global
    mean of the geopotential, i.e. the mass) is conserved."""
    print("CASE large step T1023/T511 fp64", flush=True)
    c = gold["config"]
    lf, lc = levels(pk, pk.SHX_FP64)
    st = pk.Stepper(lf, lc, niter=c["niter"], nsweep_fine=c["nsweep_fine"], nsweep_coarse=c["nsweep_coarse"])
    y = st.step(c["dt"], state)
    check(y, gold["step"], TOL, "step", gold["step_order_sensitivity"])
    assert abs(y[0, 0] - state[0, 0]).item() <= 1e-12 * torch.linalg.vector_norm(state[0]).item()


@pytest.mark.parametrize("tmode", [0, 1])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_large_mixed(pk, gold, state, prec, tmode):
    """Reduced-precision Legendre contractions at T1023/T511, with the tables
    in device memory and without: tendency within five times the emulated
    error, one step within the stated error of the FP64 oracle."""
    print("CASE large mixed", prec, "table mode", tmode, flush=True)
    with open(MIXED) as fh:
        emu = json.load(fh)["f_explicit_rel_err"][MODE_NAMES[prec]]
    c = gold["config"]
    lf, lc = levels(pk, prec, tmode)
    _, fe = pk.tendency(lf.plan, pk.swe_params(), state[None].contiguous())
    for f, rec in enumerate(gold["f_explicit"]):
        est, full = sampled_error(fe[0, f], rec)
        print("mixed tendency", prec, tmode, f, est, full, "emulated", emu[f], flush=True)
        assert est < 5.0 * emu[f] and full < 5.0 * emu[f], (f, est, full, emu[f])
    st = pk.Stepper(lf, lc, niter=c["niter"], nsweep_fine=c["nsweep_fine"], nsweep_coarse=c["nsweep_coarse"])
    y = st.step(c["dt"], state)
    for f, rec in enumerate(gold["step"]):
        est, full = sampled_error(y[f], rec)
        print("mixed step", prec, tmode, f, est, full, flush=True)
        assert est < BOUND_STEP[prec] and full < BOUND_STEP[prec], (f, est, full)
    assert np.isfinite(torch.view_as_real(y).cpu().numpy()).all()
