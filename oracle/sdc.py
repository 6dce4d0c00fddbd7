"""IMEX SDC sweep, two-level MLSDC step and collocation residual, plain FP64.

Sweep: Sec. 4.2, eq. update_equation_sdcq_discrete_form (single level) and
Sec. 4.3.1, eq. modified_update_equation_sdcq_discrete_form (with the FAS
term).  Step: Sec. 4.3.2, Algorithm 1, with the spread initialisation of
Sec. 4.3.2 and the transfer operators of Sec. 4.3.3.  FAS term: Sec. 4.3.1,
eq. tau_term_level_l+1 with tau_f = 0.

The solver is generic: a `problem` supplies evaluate(theta) -> (F_I, F_E)
and solve(b, h) -> theta solving theta - h F_I(theta) = b, and (for two
levels) restrict/interpolate in space.  The SWE problem lives in oracle.swe.

Readings of the paper used here:
  * The sweep is written in the paper's 0-to-node form.  F_I and F_E at a
    new node are evaluated from the new state (not recovered from b).
  * Algorithm 1, step C builds tau from the fine F after the fine sweep of
    step A (the FAS identity of Sec. 4.3.1 holds for that choice).
  * Step B loops over coarse nodes 1..M_c; coarse node 0 (the restricted
    initial value) is restricted and evaluated once per time step.
  * The new time-step value is the last fine node after step D of the last
    iteration (no extra sweep, no re-evaluation).
  * nsweep_fine / nsweep_coarse sweeps are done in steps A and C (the paper
    uses one of each).
Part of the test infrastructure.
"""
import torch

from .quadrature import sdc_matrices, transfer_matrix
from .sht import truncate, zero_pad


class Level:
    """One space-time level: a problem and a node set with its matrices."""

    def __init__(self, problem, kind="lobatto", nnodes=3):
        self.problem = problem
        self.mat = sdc_matrices(kind, nnodes)
        self.M = nnodes - 1
        self.Q = torch.tensor(self.mat.Q)
        self.QE = torch.tensor(self.mat.QE)
        self.QD = torch.tensor(self.mat.QD)


def _wsum(weights, arrs):
    """sum_j weights[j] * arrs[j] (weights real)."""
    out = None
    for wj, a in zip(weights, arrs):
        t = float(wj) * a
        out = t if out is None else out + t
    return out


def sweep(level: Level, dt, theta, fi, fe, tau=None):
    """One IMEX SDC sweep over the nodes of `level`.

    theta, fi, fe: lists of M+1 arrays (node 0 = initial value, read-only);
    tau: list of M+1 arrays or None.  Returns new lists.
    For m = 0..M-1:
      b = Theta^0 + dt sum_{j=0}^{M} q_{m+1,j} (F_I + F_E)^{j,(k)}
          + dt sum_{j=1}^{m} [qE_{m+1,j} dF_E^j + qD_{m+1,j} dF_I^j]
          - dt qD_{m+1,m+1} F_I^{m+1,(k)} + tau^{m+1},
      Theta^{m+1,(k+1)} = solve(b, dt qD_{m+1,m+1}), then evaluate.
    """
    M = level.M
    Q, QE, QD = level.Q, level.QE, level.QD
    p = level.problem
    f_old = [fi[j] + fe[j] for j in range(M + 1)]
    th = list(theta)
    fi_new = list(fi)
    fe_new = list(fe)
    for m in range(M):
        b = theta[0] + dt * _wsum(Q[m + 1], f_old)
        for j in range(1, m + 1):
            b = b + (dt * float(QE[m + 1, j])) * (fe_new[j] - fe[j]) \
                  + (dt * float(QD[m + 1, j])) * (fi_new[j] - fi[j])
        h = dt * float(QD[m + 1, m + 1])
        b = b - h * fi[m + 1]
        if tau is not None:
            b = b + tau[m + 1]
        th[m + 1] = p.solve(b, h)
        fi_new[m + 1], fe_new[m + 1] = p.evaluate(th[m + 1])
    return th, fi_new, fe_new


def fas_tau(fine: Level, coarse: Level, dt, fi_f, fe_f, fi_c, fe_c, restrict_space, Pi_cf):
    """tau_c = A_c(R Theta_f) - R A_f(Theta_f) with A(x) = x - dt (Q x I) F(x)
    (Sec. 4.3.1, eq. tau_term_level_l+1, tau_f = 0).  The state terms cancel,
    leaving tau_c^i = dt [sum_j (Pi Q_f)_{ij} D F_f^j - sum_j (Q_c)_{ij} F_c^j]."""
    Mf, Mc = fine.M, coarse.M
    PQ = torch.tensor(Pi_cf) @ fine.Q
    Ff = [restrict_space(fi_f[j] + fe_f[j]) for j in range(Mf + 1)]
    Fc = [fi_c[j] + fe_c[j] for j in range(Mc + 1)]
    return [dt * (_wsum(PQ[i], Ff) - _wsum(coarse.Q[i], Fc)) for i in range(Mc + 1)]


def mlsdc_step(fine: Level, coarse, dt, theta_n, niter, nsweep_fine=1, nsweep_coarse=1,
               restrict_space=None, interp_space=None, history=None):
    """One time step of two-level MLSDC (Algorithm 1), or single-level SDC
    (sweeps of step A only) when coarse is None.  Returns Theta^{n+1}.

    If `history` is a list, the fine node arrays after each iteration are
    appended to it (for diagnostics)."""
    Mf = fine.M
    pf = fine.problem
    # spread (Sec. 4.3.2): copy the initial value and its F to every fine node
    fi0, fe0 = pf.evaluate(theta_n)
    th_f = [theta_n] * (Mf + 1)
    fi_f = [fi0] * (Mf + 1)
    fe_f = [fe0] * (Mf + 1)
    if coarse is not None:
        Mc = coarse.M
        pc = coarse.problem
        Pi_cf = transfer_matrix(fine.mat, coarse.mat)     # restriction in time
        Pi_fc = transfer_matrix(coarse.mat, fine.mat)     # interpolation in time
        th_c0 = restrict_space(theta_n)
        fi_c0, fe_c0 = pc.evaluate(th_c0)
    for _ in range(niter):
        # A) fine sweep(s)
        for _s in range(nsweep_fine):
            th_f, fi_f, fe_f = sweep(fine, dt, th_f, fi_f, fe_f)
        if coarse is None:
            if history is not None:
                history.append(list(th_f))
            continue
        # B) restrict, re-evaluate, save the restriction
        th_c = [th_c0] + [None] * Mc
        fi_c = [fi_c0] + [None] * Mc
        fe_c = [fe_c0] + [None] * Mc
        for m in range(1, Mc + 1):
            th_c[m] = restrict_space(_wsum(Pi_cf[m], th_f))
            fi_c[m], fe_c[m] = pc.evaluate(th_c[m])
        th_c_t, fi_c_t, fe_c_t = list(th_c), list(fi_c), list(fe_c)
        # C) FAS correction and coarse sweep(s)
        tau = fas_tau(fine, coarse, dt, fi_f, fe_f, fi_c, fe_c, restrict_space, Pi_cf)
        for _s in range(nsweep_coarse):
            th_c, fi_c, fe_c = sweep(coarse, dt, th_c, fi_c, fe_c, tau)
        # D) interpolate the coarse corrections of Theta, F_I, F_E
        d_th = [th_c[i] - th_c_t[i] for i in range(Mc + 1)]
        d_fi = [fi_c[i] - fi_c_t[i] for i in range(Mc + 1)]
        d_fe = [fe_c[i] - fe_c_t[i] for i in range(Mc + 1)]
        for m in range(1, Mf + 1):
            th_f[m] = th_f[m] + interp_space(_wsum(Pi_fc[m], d_th))
            fi_f[m] = fi_f[m] + interp_space(_wsum(Pi_fc[m], d_fi))
            fe_f[m] = fe_f[m] + interp_space(_wsum(Pi_fc[m], d_fe))
        if history is not None:
            history.append(list(th_f))
    return th_f[Mf]


def collocation_residual(level: Level, dt, theta):
    """max_m ||Theta^0 + dt sum_j q_{m,j} F(Theta^j) - Theta^m||_2 / ||Theta^0||_2
    with F re-evaluated (Sec. 4.2, eq. collocation_problem)."""
    p = level.problem
    F = [sum(p.evaluate(t)) for t in theta]
    r = 0.0
    n0 = torch.linalg.vector_norm(theta[0]).item()
    for m in range(1, level.M + 1):
        rm = theta[0] + dt * _wsum(level.Q[m], F) - theta[m]
        r = max(r, torch.linalg.vector_norm(rm).item() / n0)
    return r


def spectral_transfer(N_f, N_c):
    """Space restriction (truncation D) and interpolation (zero-padding D^T)
    between truncations N_f > N_c (Sec. 4.3.3)."""
    def restrict(x):
        return truncate(x, N_f, N_c)

    def interp(x):
        return zero_pad(x, N_c, N_f)
    return restrict, interp


def mlsdc_step_multi(levels, dt, theta_n, niter, nsweeps, transfers, history=None):
    """One time step of multi-level MLSDC: the V-cycle that Algorithm 1 is
    the two-level case of (Sec. 4.3), for levels[0] (finest) .. levels[L-1].
    transfers[l] = (restrict_space, interp_space) between levels l and l+1;
    nsweeps[l] sweeps on level l per iteration.  Per iteration: sweep the
    finest level; going down, restrict the nodes 1..M of level l into level
    l+1, evaluate, save the restriction, form the FAS term
    tau_{l+1} = A_{l+1}(R Theta_l) - R A_l(Theta_l) + R tau_l (eq.
    tau_term_level_l+1, tau_l = 0 on the finest level) and sweep with it;
    going up, add the interpolated corrections of Theta, F_I and F_E of
    level l+1 to level l.  Node 0 of every coarser level is the restricted
    initial value, evaluated once per step.  With two levels this is
    mlsdc_step."""
    L = len(levels)
    M = [lv.M for lv in levels]
    p0 = levels[0].problem
    fi0, fe0 = p0.evaluate(theta_n)
    th = [[theta_n] * (M[0] + 1)]
    fi = [[fi0] * (M[0] + 1)]
    fe = [[fe0] * (M[0] + 1)]
    P_down, P_up, x0 = [], [], [theta_n]
    for l in range(1, L):
        P_down.append(transfer_matrix(levels[l - 1].mat, levels[l].mat))
        P_up.append(transfer_matrix(levels[l].mat, levels[l - 1].mat))
        x0.append(transfers[l - 1][0](x0[l - 1]))
    f0 = [None] + [levels[l].problem.evaluate(x0[l]) for l in range(1, L)]
    for _ in range(niter):
        for _s in range(nsweeps[0]):
            th[0], fi[0], fe[0] = sweep(levels[0], dt, th[0], fi[0], fe[0])
        saved = [None] * L
        tau = [None] * L
        del th[1:], fi[1:], fe[1:]
        for l in range(1, L):
            lv, restrict = levels[l], transfers[l - 1][0]
            t_l = [x0[l]] + [None] * M[l]
            i_l = [f0[l][0]] + [None] * M[l]
            e_l = [f0[l][1]] + [None] * M[l]
            for m in range(1, M[l] + 1):
                t_l[m] = restrict(_wsum(P_down[l - 1][m], th[l - 1]))
                i_l[m], e_l[m] = lv.problem.evaluate(t_l[m])
            saved[l] = (list(t_l), list(i_l), list(e_l))
            tau[l] = fas_tau(levels[l - 1], lv, dt, fi[l - 1], fe[l - 1], i_l, e_l, restrict, P_down[l - 1])
            if tau[l - 1] is not None:
                rt = [restrict(_wsum(P_down[l - 1][i], tau[l - 1])) for i in range(M[l] + 1)]
                tau[l] = [tau[l][i] + rt[i] for i in range(M[l] + 1)]
            for _s in range(nsweeps[l]):
                t_l, i_l, e_l = sweep(lv, dt, t_l, i_l, e_l, tau[l])
            th.append(t_l)
            fi.append(i_l)
            fe.append(e_l)
        for l in range(L - 1, 0, -1):
            interp = transfers[l - 1][1]
            st, si, se = saved[l]
            d_th = [th[l][i] - st[i] for i in range(M[l] + 1)]
            d_fi = [fi[l][i] - si[i] for i in range(M[l] + 1)]
            d_fe = [fe[l][i] - se[i] for i in range(M[l] + 1)]
            for m in range(1, M[l - 1] + 1):
                th[l - 1][m] = th[l - 1][m] + interp(_wsum(P_up[l - 1][m], d_th))
                fi[l - 1][m] = fi[l - 1][m] + interp(_wsum(P_up[l - 1][m], d_fi))
                fe[l - 1][m] = fe[l - 1][m] + interp(_wsum(P_up[l - 1][m], d_fe))
        if history is not None:
            history.append(list(th[0]))
    return th[0][M[0]]
