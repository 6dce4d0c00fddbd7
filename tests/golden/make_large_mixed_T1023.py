"""Writes tests/golden/large_T1023_mixed.json: the error of the explicit
tendency F_E at T1023 (3072 x 1536 Gaussian grid, the seeded state of the
large configuration) when the Legendre contractions run in FP32 or split
BF16 (2 or 3 pieces), as predicted by the CPU emulation oracle.mixed on the
full result: per mode and field, ||F_E(mode) - F_E(FP64)|| / ||F_E(FP64)||.
Calls only the oracle.  (About an hour on 8 cores: the emulated sums take
one FP32 accumulation step at a time.)"""
import json
import os
import sys
import time

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workload  # noqa: E402
from oracle import mixed as OM  # noqa: E402
from oracle import swe as OW  # noqa: E402


def main():
    torch.set_num_threads(max(1, os.cpu_count() or 1))
    t0 = time.time()
    fine = workload.WORKLOADS["T1023"]
    seed = workload.SEEDS["mlsdc_T1023"][0]
    prob = OW.SWEProblem(fine["N"], fine["J"], fine["I"])
    st = torch.tensor(workload.state(fine["N"], seed))
    ref = OW.f_explicit(st, prob.grid, prob.p)
    print("fp64", time.time() - t0, flush=True)
    out = {"config": {"fine": fine, "seed": seed}, "f_explicit_rel_err": {}}
    for mode in ("fp32", "bf16x2", "bf16x3"):
        fe = OW.f_explicit(st, OM.MixedGrid(prob.grid, mode), prob.p)
        out["f_explicit_rel_err"][mode] = [
            (torch.linalg.vector_norm(fe[f] - ref[f]) / torch.linalg.vector_norm(ref[f])).item() for f in range(3)]
        print(mode, out["f_explicit_rel_err"][mode], time.time() - t0, flush=True)
    with open(os.path.join(HERE, "large_T1023_mixed.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
