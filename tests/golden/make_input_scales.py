"""Writes tests/golden/input_scales.json: the factors that scale the seeded
raw spectra of workload/ to a maximum wind speed of 40 m/s and a maximum
|Phi'| of 1 % of the mean geopotential (2.94e4 m^2/s^2), both taken over the
workload's own Gaussian grid.  Calls only the oracle."""
import json
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workload  # noqa: E402
from oracle.sht import Grid  # noqa: E402
from oracle.swe import velocity_coeffs  # noqa: E402

TARGETS = {"T31": ["sdc_T31"], "T127": ["mlsdc_T127", "adjoint_T127"], "T255": ["pair_T255", "mlsdc_T255"],
           "T1023": ["mlsdc_T1023"]}


def main():
    out = {}
    path = os.path.join(HERE, "input_scales.json")
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for wl, names in TARGETS.items():
        d = workload.WORKLOADS[wl]
        N = d["N"]
        g = Grid(N, d["J"], d["I"])
        a = workload.CONSTANTS["a"]
        for name in names:
            for seed in workload.SEEDS[name]:
                raw = torch.tensor(workload.raw_spectrum(N, seed))
                U, V = velocity_coeffs(raw[1], raw[2], N, a)
                u = g.sh_inverse(U, N + 1) / g.sin_theta[:, None]
                v = g.sh_inverse(V, N + 1) / g.sin_theta[:, None]
                wmax = torch.sqrt(u * u + v * v).max().item()
                pmax = g.sh_inverse(raw[0]).abs().max().item()
                out[workload.scale_key(N, seed)] = {
                    "wind": 40.0 / wmax,
                    "phi": 0.01 * workload.CONSTANTS["phibar"] / pmax,
                }
                print(workload.scale_key(N, seed), out[workload.scale_key(N, seed)], flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
