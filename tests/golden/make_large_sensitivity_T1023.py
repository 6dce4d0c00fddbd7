"""Writes tests/golden/large_T1023_sensitivity.json: how far the FP64
oracle's explicit tendency F_E at T1023 (the seeded state of the large
configuration) moves when only the rounding of its sums changes.  Besides the
latitude order of the Legendre analysis (stored with the sampled results in
large_T1023.json), two more reorderings that any FP64 implementation may
make: the Legendre synthesis summed over the degrees in the opposite order,
and the longitude transforms computed as full-length complex FFTs instead of
real-input FFTs; and the Legendre functions themselves moved within their
last bit (every tabulated value multiplied by 1 + 2^-53 r, r uniform in
[-1, 1], seeded), the uncertainty of any FP64 table of them.  Per field:
||F_E(variant) - F_E|| / ||F_E||.  Calls only the oracle.
    python tests/golden/make_large_sensitivity_T1023.py [variant ...]
recomputes the named variants (default: all) and keeps the others stored.
The variant all_at_once makes all of these changes together and also
reverses the latitude order.  Two more replace the exactly rounded functions
by the FP64 three-term recurrence, started once per order
(fp64_recurrence) or restarted from exact values every 64 degrees
(fp64_recurrence_restart_64)."""
import json
import math
import os
import sys
import time

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workload  # noqa: E402
from oracle import sht as OH  # noqa: E402
from oracle import swe as OW  # noqa: E402


class ReversedSynthesisGrid:
    """The oracle's Grid with the sum over degrees of the synthesis taken in
    the opposite order."""

    def __init__(self, grid):
        self.__dict__.update(grid.__dict__)
        self._grid = grid

    def legendre_synthesis(self, spec, nmax=None):
        N = self.N
        nmax = N if nmax is None else nmax
        blocks = OH.split_m(spec, N, nmax)
        cols = []
        for m in range(N + 1):
            Pm = self.P[m][: nmax + 1 - m].to(OH.CT)
            cols.append(blocks[m].flip(-1) @ Pm.flip(0))
        return torch.stack(cols, dim=-1)

    def legendre_analysis(self, four, weights, nmax=None):
        return self._grid.legendre_analysis(four, weights, nmax)

    def fourier_synthesis(self, four):
        return self._grid.fourier_synthesis(four)

    def fourier_analysis(self, grid):
        return self._grid.fourier_analysis(grid)

    def sh_inverse(self, spec, nmax=None):
        return self.fourier_synthesis(self.legendre_synthesis(spec, nmax))


class ComplexFFTGrid:
    """The oracle's Grid with both longitude transforms done by full-length
    complex FFTs (the same sums as eqs. spectral_to_physical_space and
    fourier_transform, rounded differently)."""

    def __init__(self, grid):
        self.__dict__.update(grid.__dict__)
        self._grid = grid

    def legendre_synthesis(self, spec, nmax=None):
        return self._grid.legendre_synthesis(spec, nmax)

    def legendre_analysis(self, four, weights, nmax=None):
        return self._grid.legendre_analysis(four, weights, nmax)

    def fourier_synthesis(self, four):
        I, N = self.I, self.N
        full = torch.zeros(four.shape[:-1] + (I,), dtype=OH.CT)
        f0 = four.clone()
        f0[..., 0] = f0[..., 0].real.to(OH.CT)
        full[..., : N + 1] = f0
        full[..., I - N:] = f0[..., 1:].conj().flip(-1)
        return torch.fft.ifft(full, dim=-1).real * I

    def fourier_analysis(self, grid):
        return torch.fft.fft(grid.to(OH.CT), dim=-1)[..., : self.N + 1] / self.I

    def sh_inverse(self, spec, nmax=None):
        return self.fourier_synthesis(self.legendre_synthesis(spec, nmax))


class PerturbedTableGrid:
    """The oracle's Grid with every P^m_n(mu_j) moved within its last bit."""

    def __init__(self, grid, seed=11):
        self.__dict__.update(grid.__dict__)
        gen = torch.Generator().manual_seed(seed)
        self.P = [Pm * (1.0 + 2.0 ** -53 * (2.0 * torch.rand(Pm.shape, generator=gen, dtype=torch.float64) - 1.0))
                  for Pm in grid.P]

    legendre_synthesis = OH.Grid.legendre_synthesis
    legendre_analysis = OH.Grid.legendre_analysis
    fourier_synthesis = OH.Grid.fourier_synthesis
    fourier_analysis = OH.Grid.fourier_analysis
    sh_inverse = OH.Grid.sh_inverse
    sh_forward = OH.Grid.sh_forward


class RecurrenceTableGrid:
    """The oracle's Grid with P^m_n(mu_j) generated in FP64 by the three-term
    recurrence of the orthonormal functions (Sec. 3),
    P_n = (mu P_{n-1} - eps_{n-1} P_{n-2}) / eps_n, eps_n = sqrt((n^2 - m^2) / (4 n^2 - 1)),
    started from the exactly rounded values P_k, P_{k+1} at every restart
    degree k = m + r R (r = 0, 1, ...): R = restart spacing (None: started at
    n = m only), the way an on-the-fly transform generates the functions."""

    def __init__(self, grid, spacing=None):
        self.__dict__.update(grid.__dict__)
        x = grid.mu.numpy()
        out = []
        for m, Pm in enumerate(grid.P):
            P = Pm.numpy()
            Q = np.empty_like(P)
            for k in range(P.shape[0]):
                n = m + k
                if k < 2 or (spacing and k % spacing < 2):
                    Q[k] = P[k]
                else:
                    e1 = math.sqrt((n * n - m * m) / (4.0 * n * n - 1.0))
                    e0 = math.sqrt(((n - 1) ** 2 - m * m) / (4.0 * (n - 1) ** 2 - 1.0))
                    Q[k] = (x * Q[k - 1] - e0 * Q[k - 2]) / e1
            out.append(torch.from_numpy(Q))
        self.P = out

    legendre_synthesis = OH.Grid.legendre_synthesis
    legendre_analysis = OH.Grid.legendre_analysis
    fourier_synthesis = OH.Grid.fourier_synthesis
    fourier_analysis = OH.Grid.fourier_analysis
    sh_inverse = OH.Grid.sh_inverse
    sh_forward = OH.Grid.sh_forward


class AllChangesGrid:
    """All of the changes above at once, with the latitudes in reverse order
    as well (the analysis then sums south to north): how far apart two
    equally valid FP64 evaluations of the tendency may lie."""

    def __init__(self, grid):
        self.__dict__.update(grid.__dict__)
        pert = PerturbedTableGrid(grid).P
        self.P = [Pm.flip(1) for Pm in pert]
        del pert
        self.mu, self.sin_theta, self.cos2phi, self.w = (t.flip(0) for t in (grid.mu, grid.sin_theta,
                                                                               grid.cos2phi, grid.w))

    legendre_synthesis = ReversedSynthesisGrid.legendre_synthesis
    legendre_analysis = OH.Grid.legendre_analysis
    fourier_synthesis = ComplexFFTGrid.fourier_synthesis
    fourier_analysis = ComplexFFTGrid.fourier_analysis
    sh_inverse = OH.Grid.sh_inverse
    sh_forward = OH.Grid.sh_forward


def main():
    torch.set_num_threads(max(1, os.cpu_count() or 1))
    t0 = time.time()
    fine = workload.WORKLOADS["T1023"]
    seed = workload.SEEDS["mlsdc_T1023"][0]
    prob = OW.SWEProblem(fine["N"], fine["J"], fine["I"])
    st = torch.tensor(workload.state(fine["N"], seed))
    ref = OW.f_explicit(st, prob.grid, prob.p)
    path = os.path.join(HERE, "large_T1023_sensitivity.json")
    out = {"config": {"fine": fine, "seed": seed}}
    if os.path.exists(path):
        with open(path) as f:
            out.update(json.load(f))
    variants = {"synthesis_degree_order": ReversedSynthesisGrid, "complex_fft": ComplexFFTGrid,
                "table_last_bit": PerturbedTableGrid, "all_at_once": AllChangesGrid,
                "fp64_recurrence": RecurrenceTableGrid,
                "fp64_recurrence_restart_64": lambda g: RecurrenceTableGrid(g, 64)}
    for name in sys.argv[1:] or list(variants):
        g = variants[name](prob.grid)
        fe = OW.f_explicit(st, g, prob.p)
        del g
        out[name] = [(torch.linalg.vector_norm(fe[f] - ref[f]) / torch.linalg.vector_norm(ref[f])).item()
                     for f in range(3)]
        print(name, out[name], time.time() - t0, flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
