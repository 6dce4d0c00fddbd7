"""Writes adjoint_jvp.json: directional derivatives of the adjoint test loss
L = 1/2 sum_n [|Phi'^0_n|^2 + 2 sum_{m>=1} |Phi'^m_n|^2] at the final state
of an MLSDC integration, along seeded perturbations d of the initial
vorticity, by forward-mode differentiation (torch.func.jvp) through the FP64
oracle only:  dL_k = <J d_k, dL/dTheta(T)> = sum_n w Re(conj Phi' dPhi').
These are the left-hand sides of the whole-step dot-product identity
<J d, w> = <d, J^T w> that the GPU adjoint's gradient must reproduce.

    python tests/golden/make_adjoint_jvp.py   (about 5 minutes on 8 cores)
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_jvp.json")

CONFIGS = {
    # two-level Gauss-Lobatto 5/3, 2 fine + 2 coarse sweeps x 4 iterations
    "T31_T15_3steps": dict(fine=(31, 48, 96), coarse=(15, 24, 48), dt=600.0, nsteps=3, seed_state=1000,
                           seed_dirs=3000, ndirs=32),
    "T127_T63_1step": dict(fine=(127, 192, 384), coarse=(63, 96, 192), dt=300.0, nsteps=1, seed_state=1003,
                           seed_dirs=3000, ndirs=8),
}


def _work(args):
    name, k = args
    import torch
    torch.set_num_threads(1)
    import workload
    from oracle import sdc as OS
    from oracle import sht as OH
    from oracle import swe as OW
    c = CONFIGS[name]
    N, Nc = c["fine"][0], c["coarse"][0]
    lf = OS.Level(OW.SWEProblem(*c["fine"]), "lobatto", 5)
    lc = OS.Level(OW.SWEProblem(*c["coarse"]), "lobatto", 3)
    R, P = OS.spectral_transfer(N, Nc)
    th0 = torch.tensor(workload.state(N, c["seed_state"]))
    dirs = workload.directions(N, c["ndirs"], c["seed_dirs"], float(torch.linalg.vector_norm(th0[1])))
    d = torch.zeros_like(th0)
    d[1] = torch.tensor(dirs[k])

    def integrate(x):
        for _ in range(c["nsteps"]):
            x = OS.mlsdc_step(lf, lc, c["dt"], x, niter=4, nsweep_fine=2, nsweep_coarse=2, restrict_space=R,
                              interp_space=P)
        return x

    y, yd = torch.func.jvp(integrate, (th0,), (d,))
    w = torch.where(OH.orders(N) == 0, 1.0, 2.0).to(torch.float64)
    dl = (w * (y[0].real * yd[0].real + y[0].imag * yd[0].imag)).sum().item()
    return name, k, dl


def main():
    jobs = [(name, k) for name, c in CONFIGS.items() for k in range(c["ndirs"])]
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(_work, jobs, chunksize=1)
    out = {name: dict(c, fine=list(c["fine"]), coarse=list(c["coarse"]), dL=[0.0] * c["ndirs"])
           for name, c in CONFIGS.items()}
    for name, k, dl in res:
        out[name]["dL"][k] = dl
    out["_about"] = ("forward-mode directional derivatives of L along workload.directions(N, ndirs, seed_dirs, "
                     "||zeta^0||) applied to the initial vorticity, through the FP64 oracle (torch.func.jvp); "
                     "written by tests/golden/make_adjoint_jvp.py")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
