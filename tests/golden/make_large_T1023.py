"""Writes tests/golden/large_T1023.json: sampled FP64 oracle results for the
large two-level configuration (fine T1023 on the 3072 x 1536 Gaussian grid
with 5 Gauss-Radau-right collocation points, coarse T511 on 1536 x 768 with
3; 2 fine + 2 coarse sweeps per iteration, 4 iterations, dt = 60 s), whose
full-size oracle runs take minutes.  Calls only the oracle.

Stored per field: the 2-norm of the full result and the values at seeded
sample positions, for
  * the synthesis of the seeded T1023 state (grid samples),
  * the analysis of the pointwise square of that grid (spectral samples),
  * the explicit tendency F_E of the state (spectral samples),
  * one MLSDC step from the state (spectral samples).
For the tendency and the step it also stores, per field, the oracle's own
sensitivity to the order of its latitude sums: the normwise relative
difference between the oracle and the same oracle with the latitudes taken
south to north (the Legendre analysis is the only sum over latitudes, so this
changes nothing but its rounding)."""
import copy
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workload  # noqa: E402
from oracle import sdc as OS  # noqa: E402
from oracle import sht as OH  # noqa: E402
from oracle import swe as OW  # noqa: E402

NS = 512          # samples per field
DT = 60.0
NITER, NSF, NSC = 4, 2, 2
NODES_F, NODES_C = 6, 4   # tau_0 plus 5 (fine) and 3 (coarse) Radau-IIA points


def sample_positions(n_total, seed):
    return np.sort(np.random.default_rng(seed).choice(n_total, size=NS, replace=False)).tolist()


def pack_spec(x, seed):
    out = []
    for f in range(x.shape[0]):
        idx = sample_positions(x.shape[1], seed + f)
        v = x[f, idx]
        out.append({"norm": torch.linalg.vector_norm(x[f]).item(), "idx": idx,
                    "re": v.real.tolist(), "im": v.imag.tolist()})
    return out


def pack_grid(x, seed):
    out = []
    for f in range(x.shape[0]):
        flat = x[f].reshape(-1)
        idx = sample_positions(flat.numel(), seed + f)
        out.append({"norm": torch.linalg.vector_norm(flat).item(), "idx": idx, "val": flat[idx].tolist()})
    return out


def reversed_grid(g):
    r = copy.copy(g)
    r.mu, r.sin_theta, r.cos2phi, r.w = g.mu.flip(0), g.sin_theta.flip(0), g.cos2phi.flip(0), g.w.flip(0)
    r.P = [P.flip(1) for P in g.P]
    return r


def reversed_problem(prob):
    r = copy.copy(prob)
    r.grid = reversed_grid(prob.grid)
    return r


def sensitivity(x, y):
    return [(torch.linalg.vector_norm(x[f] - y[f]) / torch.linalg.vector_norm(x[f])).item() for f in range(x.shape[0])]


def main():
    torch.set_num_threads(max(1, os.cpu_count() or 1))
    t0 = time.time()
    fine = workload.WORKLOADS["T1023"]
    coarse = workload.WORKLOADS["T511"]
    seed = workload.SEEDS["mlsdc_T1023"][0]
    pf = OW.SWEProblem(fine["N"], fine["J"], fine["I"])
    pc = OW.SWEProblem(coarse["N"], coarse["J"], coarse["I"])
    print("grids", time.time() - t0, flush=True)
    st = torch.tensor(workload.state(fine["N"], seed))
    out = {"config": {"fine": fine, "coarse": coarse, "kind": "radau", "nodes_fine": NODES_F,
                      "nodes_coarse": NODES_C, "dt": DT, "niter": NITER, "nsweep_fine": NSF,
                      "nsweep_coarse": NSC, "seed": seed, "samples_per_field": NS}}
    grid = pf.grid.sh_inverse(st)
    out["synthesis"] = pack_grid(grid, 5000)
    out["analysis_of_square"] = pack_spec(pf.grid.sh_forward(grid * grid), 5100)
    fe = OW.f_explicit(st, pf.grid, pf.p)
    out["f_explicit"] = pack_spec(fe, 5200)
    out["f_explicit_order_sensitivity"] = sensitivity(fe, OW.f_explicit(st, reversed_grid(pf.grid), pf.p))
    print("pair + tendency", time.time() - t0, flush=True)
    lf = OS.Level(pf, "radau", NODES_F)
    lc = OS.Level(pc, "radau", NODES_C)
    R, P = OS.spectral_transfer(fine["N"], coarse["N"])
    y = OS.mlsdc_step(lf, lc, DT, st, niter=NITER, nsweep_fine=NSF, nsweep_coarse=NSC, restrict_space=R,
                      interp_space=P)
    out["step"] = pack_spec(y, 5300)
    out["evaluations"] = {"fine": pf.n_eval, "coarse": pc.n_eval}
    print("step", time.time() - t0, pf.n_eval, pc.n_eval, flush=True)
    lfr = OS.Level(reversed_problem(pf), "radau", NODES_F)
    lcr = OS.Level(reversed_problem(pc), "radau", NODES_C)
    yr = OS.mlsdc_step(lfr, lcr, DT, st, niter=NITER, nsweep_fine=NSF, nsweep_coarse=NSC, restrict_space=R,
                       interp_space=P)
    out["step_order_sensitivity"] = sensitivity(y, yr)
    print("sensitivity", out["f_explicit_order_sensitivity"], out["step_order_sensitivity"], flush=True)
    with open(os.path.join(HERE, "large_T1023.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
