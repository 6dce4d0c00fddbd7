"""CPU emulation of the reduced-precision Legendre contractions.

The FP64 oracle (oracle.sht) defines the exact results; this module predicts
the error level of computing the Legendre step of eqs. spectral_to_physical_space
and legendre_transform (Sec. 3) with
  'fp32'    : table and operand rounded to FP32, FP32 accumulation;
  'bf16x2'  : x = x_hi + x_lo (bf16 pieces), products hi*hi + hi*lo + lo*hi,
              FP32 accumulation;
  'bf16x3'  : x = x_hi + x_mid + x_lo, the six products whose piece orders sum
              to at most 2, FP32 accumulation.
FP32 accumulation is recursive summation over the contraction index in its
natural order (latitudes north to south, degrees upwards): every step adds
the exact product to the running FP32 sum and rounds once, as a fused
multiply-add does.  (A library FP32 matmul keeps several partial sums in an
unstated blocking and so predicts a smaller error than a single accumulator
chain.)  In the split modes the leading product and the corrections are
accumulated in two such chains and added in FP64.  bf16 pieces come from
torch.bfloat16 (round to nearest even).  The emulation is not bitwise equal
to the GPU (the order of the sums differs); the tests use it to check that
the GPU error is of the predicted size.
Part of the test infrastructure.
"""
import numpy as np
import torch

from .sht import CT, DT, split_m


def split(x, nterms):
    """Pieces of a float64 tensor: bf16-rounded remainders (as float32 tensors)."""
    out, rem = [], x.clone()
    for _ in range(nterms):
        h = rem.to(torch.float32).to(torch.bfloat16).to(torch.float32)
        out.append(h)
        rem = rem - h.to(DT)
    return out


def accumulate_f32(T):
    """sum_k T[k] for an exact FP64 array T [K, R, C] (numpy), accumulated in
    FP32: s <- fl32(s + T[k]) in the order k = 0, 1, ....  (The FP64 addition
    before the rounding to FP32 can round once more; that changes a result by
    at most one FP32 unit in rare cases, which does not matter for an error
    level.)"""
    acc = T[0].astype(np.float32)
    for k in range(1, T.shape[0]):
        acc = (acc + T[k]).astype(np.float32)                  # float32 + float64 adds in FP64
    return acc.astype(np.float64)


def mixed_matmul(A, B, mode):
    """A @ B for real float64 A [R, K], B [K, C], emulating the
    reduced-precision contraction over K."""
    if A.shape[1] == 0:
        return torch.zeros(A.shape[0], B.shape[1], dtype=DT)
    if mode == "fp32":
        a = A.to(torch.float32).to(DT).numpy()
        b = B.to(torch.float32).to(DT).numpy()
        return torch.from_numpy(accumulate_f32(a.T[:, :, None] * b[:, None, :]))   # exact products
    n = 2 if mode == "bf16x2" else 3
    a = [x.to(DT).numpy().T[:, :, None] for x in split(A, n)]
    b = [x.to(DT).numpy()[:, None, :] for x in split(B, n)]
    pairs = [(0, 1), (1, 0)] + ([(0, 2), (2, 0), (1, 1)] if n == 3 else [])
    lead = accumulate_f32(a[0] * b[0])
    corr = accumulate_f32(sum(a[i] * b[j] for i, j in pairs))
    return torch.from_numpy(lead + corr)


def _cmatmul(A_real, Z, mode):
    """A_real @ Z for complex Z: real and imaginary parts contracted as
    separate columns."""
    C = Z.shape[1]
    out = mixed_matmul(A_real, torch.cat([Z.real, Z.imag], dim=1).contiguous(), mode)
    return torch.complex(out[:, :C], out[:, C:])


def legendre_synthesis(grid, spec, mode, nmax=None):
    """spec [F, nspec(N, nmax)] -> Fourier [F, J, N+1] in reduced precision."""
    N = grid.N
    nmax = N if nmax is None else nmax
    blocks = split_m(spec, N, nmax)
    cols = []
    for m in range(N + 1):
        Pm = grid.P[m][: nmax + 1 - m]                       # (deg, J) float64
        cols.append(_cmatmul(Pm.transpose(0, 1).contiguous(), blocks[m].transpose(0, 1), mode).transpose(0, 1))
    return torch.stack(cols, dim=-1)


def legendre_analysis(grid, four, weights, mode, nmax=None):
    """Fourier [F, J, N+1] (weights applied here) -> spec [F, nspec(N, nmax)]."""
    N = grid.N
    nmax = N if nmax is None else nmax
    out = []
    for m in range(N + 1):
        Pm = grid.P[m][: nmax + 1 - m]                       # (deg, J)
        g = (four[..., :, m] * weights.to(CT)).transpose(0, 1)   # (J, F)
        out.append(_cmatmul(Pm.contiguous(), g.contiguous(), mode).transpose(0, 1))
    return torch.cat(out, dim=-1)


def sh_inverse(grid, spec, mode):
    return grid.fourier_synthesis(legendre_synthesis(grid, spec, mode))


def sh_forward(grid, gridvals, mode):
    return legendre_analysis(grid, grid.fourier_analysis(gridvals), grid.w, mode)


class MixedGrid:
    """The oracle's Grid with its Legendre steps emulated in `mode` (the
    Fourier steps and everything else stay FP64), so that the oracle's
    tendency (oracle.swe.f_explicit) run on it predicts the error of a
    reduced-precision plan's tendency."""

    def __init__(self, grid, mode):
        self.__dict__.update(grid.__dict__)
        self._grid, self.mode = grid, mode

    def legendre_synthesis(self, spec, nmax=None):
        if spec.dim() == 1:                              # one field: [nspec] -> [J, N+1]
            return legendre_synthesis(self._grid, spec[None], self.mode, nmax)[0]
        return legendre_synthesis(self._grid, spec, self.mode, nmax)

    def legendre_analysis(self, four, weights, nmax=None):
        if four.dim() == 2:                              # one field: [J, N+1] -> [nspec]
            return legendre_analysis(self._grid, four[None], weights, self.mode, nmax)[0]
        return legendre_analysis(self._grid, four, weights, self.mode, nmax)

    def fourier_synthesis(self, four):
        return self._grid.fourier_synthesis(four)

    def fourier_analysis(self, grid):
        return self._grid.fourier_analysis(grid)

    def sh_inverse(self, spec, nmax=None):
        return self.fourier_synthesis(self.legendre_synthesis(spec, nmax))

    def sh_forward(self, grid, nmax=None):
        return self.legendre_analysis(self.fourier_analysis(grid), self.w, nmax)
