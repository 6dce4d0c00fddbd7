"""CPU emulation of the reduced-precision Legendre contractions.

The FP64 oracle (oracle.sht) defines the exact results; this module predicts
the error level of computing the Legendre step of eqs. spectral_to_physical_space
and legendre_transform (Sec. 3) with
  'fp32'    : table and operand rounded to FP32, FP32 accumulation;
  'bf16x2'  : x = x_hi + x_lo (bf16 pieces), products hi*hi + hi*lo + lo*hi,
              FP32 accumulation;
  'bf16x3'  : x = x_hi + x_mid + x_lo, the six products whose piece orders sum
              to at most 2, FP32 accumulation.
The leading product and the corrections are accumulated separately and added
in FP64.  bf16 pieces come from torch.bfloat16 (round to nearest even).  The
emulation is not bitwise equal to the GPU (summation order differs); the tests
use it to check that the GPU error is of the predicted size.
Part of the test infrastructure.
"""
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


def mixed_matmul(A, B, mode):
    """A @ B for real float64 A, B, emulating the reduced-precision contraction."""
    if mode == "fp32":
        return (A.to(torch.float32) @ B.to(torch.float32)).to(DT)
    n = 2 if mode == "bf16x2" else 3
    a, b = split(A, n), split(B, n)
    lead = (a[0] @ b[0]).to(DT)
    corr = a[0] @ b[1] + a[1] @ b[0]
    if n == 3:
        corr = corr + a[0] @ b[2] + a[2] @ b[0] + a[1] @ b[1]
    return lead + corr.to(DT)


def _cmatmul(A_real, Z, mode):
    """A_real @ Z for complex Z: real and imaginary parts contracted separately."""
    return torch.complex(mixed_matmul(A_real, Z.real.contiguous(), mode),
                         mixed_matmul(A_real, Z.imag.contiguous(), mode))


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
