"""mlsdc_step_noalloc, the allocation-free variant of mlsdc_step (its
workspace is the library's per-device scratch array), called through the C
ABI and compared with mlsdc_step on the same inputs: two calls in a row, the
second on a smaller configuration, each bit-identical to mlsdc_step (the same
kernels on the same data); a configuration beyond the scratch limit is
rejected before anything is enqueued."""
import ctypes

import pytest
import torch

import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07923_amd as pk
    pk.lib()
    return pk


def _level(pk, N, J, I, nn, par):
    return pk.Level(pk.Plan(N, J, I), par, pk.SDC_GAUSS_LOBATTO, nn)


def test_noalloc_matches_mlsdc_step(pk):
    par = pk.swe_params()
    cases = [
        # fine, coarse, niter, sweeps (fine, coarse), dt, seed: the T255/T127 step, then a smaller one
        ((255, 384, 768, 5), (127, 192, 384, 3), 4, (2, 2), 300.0, 1005),
        ((31, 48, 96, 3), (15, 24, 48, 2), 2, (1, 1), 600.0, 1000),
    ]
    for fs, cs, niter, (nsf, nsc), dt, seed in cases:
        print("CASE noalloc", fs, cs, niter, nsf, nsc, flush=True)
        lf, lc = _level(pk, *fs, par), _level(pk, *cs, par)
        stepper = pk.Stepper(lf, lc, niter=niter, nsweep_fine=nsf, nsweep_coarse=nsc)
        print("workspace bytes", stepper.nbytes, flush=True)
        assert stepper.nbytes <= 96 * 1024 * 1024
        x = torch.tensor(workload.state(fs[0], seed)).cuda()
        ref = stepper.step(dt, x)
        st_ref = torch.zeros(2, dtype=torch.float64, device="cuda")
        ref2 = stepper.step(dt, x, status=st_ref)
        out = torch.full_like(x, float("nan"))
        st = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        got = stepper.step_noalloc(dt, x, out, status=st)
        torch.cuda.synchronize()
        assert got is out
        assert torch.equal(out, ref) and torch.equal(ref2, ref)
        assert torch.equal(st, st_ref)
        assert torch.isfinite(out).all()


def test_noalloc_rejects_beyond_scratch(pk):
    """The T255/T127 step with the residual check needs more than the scratch
    limit: SHX_EWORKSPACE, and the output is untouched."""
    par = pk.swe_params()
    lf = _level(pk, 255, 384, 768, 5, par)
    lc = _level(pk, 127, 192, 384, 3, par)
    opts = pk.MlsdcOpts(4, 2, 2, 1)
    need = pk.lib().mlsdc_workspace_bytes(lf.h, lc.h, ctypes.byref(opts))
    assert need > 96 * 1024 * 1024
    x = torch.tensor(workload.state(255, 1005)).cuda()
    out = torch.zeros_like(x)
    rc = pk.lib().mlsdc_step_noalloc(lf.h, lc.h, ctypes.byref(opts), 300.0, x.data_ptr(), out.data_ptr(), None,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == -4
    assert torch.count_nonzero(out).item() == 0
