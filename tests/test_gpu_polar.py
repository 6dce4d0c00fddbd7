"""Polar truncation of the table analyses (the near-pole omission of the
transform library the method builds on, Sec. 3, Schaeffer 2013).

FP64 and FP32 plans with tables on at most 512 latitudes leave out of the Legendre
analysis, per order, parity and 16-degree tile, the groups of 4 latitude
pairs nearest the pole for as long as every |P^m_n| of the group is below
1e-20, less the groups that make the summed run whole batches of loads
(8 groups from 160 latitude pairs up, 4 below).  Two checks:
  * the number of summed table products that the plan reports equals the
    count the same rule gives on the oracle's P^m_n (bracketed by the rule at
    1e-20 (1 -+ 1e-9), so that values within rounding of the threshold may
    fall either way), and the plan without tables sums every pair;
  * the analysis of fields that live only near the poles, where all omitted
    terms are, matches the oracle's full sums coefficient by coefficient
    (an omitted group holding a value above the threshold would show here).
"""
import numpy as np
import pytest
import torch

from oracle import quadrature as OQ
from oracle import sht as OH

pytestmark = pytest.mark.gpu

TAU = 1e-20


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07923_amd as pk
    pk.lib()
    return pk


def rule_counts(N, J, nmax, tau):
    """(products, Fourier (m, pair) rows) of the truncated analysis under the
    documented rule, from the oracle's P^m_n."""
    Jh = J // 2
    ngrp, B = (Jh + 3) // 4, (8 if Jh >= 160 else 4)
    mu, st, _, _ = OQ.gauss_legendre(J)
    terms = rows = 0
    for m in range(N + 1):
        P = np.abs(OH.legendre_m(m, nmax, mu[:Jh], st[:Jh]))      # degrees m..nmax
        first = Jh
        for p in (0, 1):
            blk = P[p::2]
            for kt in range(0, blk.shape[0], 16):
                tile = blk[kt:kt + 16]
                big = np.nonzero(tile.max(axis=0) >= tau)[0]
                c0 = big[0] // 4 if len(big) else ngrp
                cs = max(0, ngrp - B * (-(-(ngrp - c0) // B)))   # whole batches of B groups
                j0 = min(4 * cs, Jh)
                terms += tile.shape[0] * (Jh - j0)
                first = min(first, j0)
        rows += Jh - first
    return terms, rows


@pytest.mark.parametrize("N,J,I", [(31, 48, 96), (127, 192, 384), (255, 384, 768)])
def test_polar_terms_follow_the_rule(pk, N, J, I):
    print("CASE polar terms", N, J, I, flush=True)
    full = sum(((N + 1 - m - p) // 2 + 1) * (J // 2) for m in range(N + 1) for p in (0, 1)
               if N + 1 - m - p >= 0)
    plan = pk.Plan(N, J, I)
    terms, rows = plan.analysis_terms(N + 1)
    lo_t, lo_r = rule_counts(N, J, N + 1, TAU * (1 + 1e-9))
    hi_t, hi_r = rule_counts(N, J, N + 1, TAU * (1 - 1e-9))
    assert lo_t <= terms <= hi_t, (terms, lo_t, hi_t)
    assert lo_r <= rows <= hi_r, (rows, lo_r, hi_r)
    if N == 255:
        assert terms < 0.95 * full                  # the truncation does take effect at T255
    otf = pk.Plan(N, J, I, table_mode=pk.SHX_TABLE_ONTHEFLY)
    assert otf.analysis_terms(N + 1) == (full, (N + 1) * (J // 2))
    # FP32 plans with tables truncate their FP32 tiles by the same rule
    t32, r32 = pk.Plan(N, J, I, pk.SHX_FP32).analysis_terms(N + 1)
    assert lo_t <= t32 <= hi_t and lo_r <= r32 <= hi_r, (t32, r32)


@pytest.mark.parametrize("N,J,I", [(127, 192, 384), (255, 384, 768)])
def test_polar_fields_match_full_sums(pk, N, J, I):
    """Random grid values only where |mu| > 0.8 (both caps), five fields in one
    launch; every coefficient against the oracle's full sum, to 1e-13 of the
    field's largest coefficient."""
    print("CASE polar fields", N, J, I, flush=True)
    g = OH.Grid(N, J, I)
    mu = torch.as_tensor(OQ.gauss_legendre(J)[0])
    gen = torch.Generator().manual_seed(1805)
    grid = torch.randn(5, J, I, dtype=torch.float64, generator=gen)
    grid = grid * (mu.abs() > 0.8).to(torch.float64)[None, :, None]
    plan = pk.Plan(N, J, I)
    got = plan.forward(grid.to("cuda").contiguous()).cpu()
    for f in range(5):
        ref = g.sh_forward(grid[f])
        err = (got[f] - ref).abs().max().item()
        assert err <= 1e-13 * ref.abs().max().item(), (f, err)
