// C ABI entry points: plan and level set-up, the SH transform pair, the
// shallow-water tendency, the implicit solve, the IMEX SDC sweep and the
// two-level MLSDC step (Algorithm 1).  Host code only enqueues kernels on the
// caller's stream; argument checks happen before anything is enqueued.
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"
#include "setup_host.h"

namespace {

inline hipStream_t S(shx_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

template <class T>
hipError_t dalloc(T** p, size_t n) {
    return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T) > 0 ? n * sizeof(T) : 1);
}

void plan_free(shx_plan* p) {
    if (!p) return;
    (void)hipFree(p->mu);
    (void)hipFree(p->sint);
    (void)hipFree(p->cos2);
    (void)hipFree(p->w);
    (void)hipFree(p->tw);
    (void)hipFree(p->psyn);
    (void)hipFree(p->pan);
    (void)hipFree(p->pan4);
    (void)hipFree(p->pan4f);
    (void)hipFree(p->off4);
    (void)hipFree(p->an_c0);
    (void)hipFree(p->psyn32);
    (void)hipFree(p->pan32);
    (void)hipFree(p->an16);
    (void)hipFree(p->syn16);
    (void)hipFree(p->off_an16);
    (void)hipFree(p->off_syn16);
    (void)hipFree(p->off);
    (void)hipFree(p->ck);
    (void)hipFree(p->ckoff);
    (void)hipFree(p->rc);
    (void)hipFree(p->rq);
    (void)hipFree(p->cs);
    (void)hipFree(p->pf);
    (void)hipFree(p->ninv);
    (void)hipFree(p->nn1);
    (void)hipFree(p->anblk);
    (void)hipFree(p->tblk);
    (void)hipFree(p->ord);
    (void)hipFree(p->deg);
    (void)hipFree(p->ord_e);
    (void)hipFree(p->deg_e);
    delete p;
}

#define HIPCHK(x)                          \
    do {                                   \
        if ((x) != hipSuccess) return SHX_EHIP; \
    } while (0)

// Workspace carve-up helper.
struct Carve {
    char* base;
    size_t used = 0;
    template <class T>
    T* take(size_t n) {
        T* r = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += align256(n * sizeof(T));
        return r;
    }
};

// Tendency workspace for S states: FI [S][J][N+1][4], G [S][J][N+1][5],
// cout [S][ext][5] (double2).
struct TendWS {
    double2 *FI, *G, *cout;
};
TendWS carve_tend(Carve& c, const shx_plan* pl, int S) {
    TendWS t;
    t.FI = c.take<double2>((size_t)S * pl->J * (pl->N + 1) * 4);
    t.G = c.take<double2>((size_t)S * pl->J * (pl->N + 1) * 5);
    t.cout = c.take<double2>((size_t)S * pl->nspec_e * 5);
    return t;
}
size_t tend_bytes(const shx_plan* pl, int S) {
    Carve c{nullptr};
    carve_tend(c, pl, S);
    return c.used;
}

bool alias_free(const shx_plan* pl) {
    return pl->I >= 3 * pl->N + 1 && 2 * pl->J >= 3 * pl->N + 1;
}

// Kernel timer (profiling hook): events recorded on the launch stream around
// each launch of one kernel class.  Process-global, not thread safe.
struct KernelTimer {
    int kclass = -1, cap = 0, n = 0;
    std::vector<hipEvent_t> ev0, ev1;
} g_timer;

template <class F>
hipError_t timed(int kclass, hipStream_t st, F launch) {
    const bool on = g_timer.kclass == kclass && g_timer.n < g_timer.cap;
    if (on && hipEventRecord(g_timer.ev0[g_timer.n], st) != hipSuccess) return hipErrorUnknown;
    hipError_t e = launch();
    if (on && e == hipSuccess) {
        e = hipEventRecord(g_timer.ev1[g_timer.n], st);
        ++g_timer.n;
    }
    return e;
}

// combine = false leaves F_E, F_I unformed: the analyses stay in t.cout.
int tendency_impl(const shx_plan* pl, const swe_params& p, int nst, const double2* state, double2* fi,
                  double2* fe, const TendWS& t, hipStream_t st, bool combine = true) {
    if (fe) {
        HIPCHK(timed(SHX_KC_LEGENDRE_SYN, st, [&] { return launch_leg_syn_swe(pl, p.a, state, t.FI, nst, st); }));
        HIPCHK(timed(SHX_KC_GRID, st, [&] { return launch_swe_grid(pl, t.FI, t.G, nst, p.omega, st); }));
        HIPCHK(timed(SHX_KC_LEGENDRE_AN, st, [&] { return launch_leg_an(pl, t.G, t.cout, 5, nst, pl->nmax, st); }));
    }
    if (combine) HIPCHK(launch_swe_combine(pl, p, t.cout, state, fi, fe, nst, st));
    return SHX_OK;
}

// One IMEX SDC sweep reading F_I, F_E of the previous iterate at every node
// from (fi_old, fe_old) and writing the new F at nodes 1..M to (fi_new,
// fe_new); Theta is updated in place (node 0 read only).  Node 0 of the new
// buffers is not touched.
// form_last = false leaves the F of node M unformed (its analyses stay in
// t.cout) for a following sweep on the same level, whose first update forms
// it (old_last_from_cout = true); only that update reads it.
int sweep_impl(const sdc_level* lv, double dt, double2* th, const double2* fi_old, const double2* fe_old,
               double2* fi_new, double2* fe_new, const double2* tau, const TendWS& t, hipStream_t st,
               double2* rec = nullptr, bool form_last = true, bool old_last_from_cout = false) {
    const shx_plan* pl = lv->plan;
    const int M = lv->nnodes - 1, n1 = lv->nnodes;
    const size_t ns3 = 3 * (size_t)pl->nspec;
    NodeRows rows{};
    for (int m = 0; m < M; ++m) {
        for (int j = 0; j < n1; ++j) {
            rows.q[m][j] = dt * lv->Q[(m + 1) * n1 + j];
            rows.qe[m][j] = dt * lv->QE[(m + 1) * n1 + j];
            rows.qd[m][j] = dt * lv->QD[(m + 1) * n1 + j];
        }
        rows.h[m] = dt * lv->QD[(m + 1) * n1 + (m + 1)];
    }
    for (int m = 0; m < M; ++m) {
        NodeWeights wt;
        for (int j = 0; j < 9; ++j) {
            wt.q[j] = j < n1 ? rows.q[m][j] : 0.0;
            wt.qe[j] = j < n1 ? rows.qe[m][j] : 0.0;
            wt.qd[j] = j < n1 ? rows.qd[m][j] : 0.0;
        }
        double2* r = rec ? rec + (size_t)m * ns3 : nullptr;
        const size_t o = (size_t)(m + 1) * ns3;
        if (m > 0 && leg_syn_swe_node_supported(pl) && pl->Jh < 384) {
            // node m's update (F of node m from t.cout, Theta^{m+1}) formed
            // in the staging of the synthesis of Theta^{m+1} (below
            // 384 latitude pairs: with more, the 4+ latitude-group blocks of
            // an order repeating the order's update cost more than the
            // separate launch; T1023 22.5 -> 19.9 steps/s)
            NodeFuse nf;
            nf.m = m;
            nf.h = rows.h[m];
            nf.wt = wt;
            nf.p = lv->p;
            nf.cout = t.cout;
            nf.theta = th;
            nf.fi = fi_new;
            nf.fe = fe_new;
            nf.rec = r;
            HIPCHK(timed(SHX_KC_LEGENDRE_SYN, st, [&] { return launch_leg_syn_swe_node(pl, nf, t.FI, st); }));
            HIPCHK(timed(SHX_KC_GRID, st, [&] { return launch_swe_grid(pl, t.FI, t.G, 1, lv->p.omega, st); }));
            HIPCHK(timed(SHX_KC_LEGENDRE_AN, st, [&] { return launch_leg_an(pl, t.G, t.cout, 5, 1, pl->nmax, st); }));
            continue;
        }
        // the first update forms the old-F part of every node's right-hand
        // side (held in fe_new at nodes 2..M until those are written); the
        // F of node m (m >= 1) is formed inside node m's update from t.cout
        HIPCHK(timed(SHX_KC_SDC_NODE, st, [&] {
            return m == 0 ? launch_sdc_node_first(pl, lv->p, M, rows, th, fi_old, fe_old,
                                                  old_last_from_cout ? t.cout : nullptr, tau, fe_new, r, st)
                          : launch_sdc_node(pl, lv->p, m, M, wt, rows.h[m], th, fi_new, fe_new, t.cout, r, st);
        }));
        int rc = tendency_impl(pl, lv->p, 1, th + o, fi_new + o, fe_new + o, t, st, false);
        if (rc) return rc;
    }
    const size_t oM = (size_t)M * ns3;
    if (form_last) HIPCHK(launch_swe_combine(pl, lv->p, t.cout, th + oM, fi_new + oM, fe_new + oM, 1, st));
    return SHX_OK;
}

// Workspace of the in-place sdc_sweep entry point: a copy of the caller's F.
struct SweepWS {
    double2 *fi_old, *fe_old;
    TendWS t;
};
SweepWS carve_sweep(Carve& c, const sdc_level* lv) {
    SweepWS w;
    const size_t n = (size_t)lv->nnodes * 3 * lv->plan->nspec;
    w.fi_old = c.take<double2>(n);
    w.fe_old = c.take<double2>(n);
    w.t = carve_tend(c, lv->plan, 1);
    return w;
}

Mat9x9 to_mat(const double* a, int n) {
    Mat9x9 r;
    std::memset(&r, 0, sizeof(r));
    for (int i = 0; i < n; ++i) r.a[i] = a[i];
    return r;
}

// MLSDC workspace.  Fine F in two buffers used alternately by the sweeps
// (old -> new); coarse F: the values at the restricted states (saved for the
// FAS term and step D) and two sweep buffers.
struct StepWS {
    double2 *thf, *fif[2], *fef[2];                     // fine [Mf+1][3][nsf]
    double2 *thc, *thct, *fict, *fect, *fic[2], *fec[2], *tau;  // coarse [Mc+1][3][nsc]
    double2 *rfi, *rfe;                                 // residual re-evaluation [Mf+1][3][nsf]
    double* partial;
    TendWS tf;                                          // fine, 1 state
    TendWS tc;                                          // coarse, Mc states
    TendWS tr;                                          // fine, Mf+1 states (residual)
};
StepWS carve_step(Carve& c, const sdc_level* f, const sdc_level* cl, const mlsdc_opts* o) {
    StepWS w{};
    const size_t nf = (size_t)f->nnodes * 3 * f->plan->nspec;
    w.thf = c.take<double2>(nf);
    for (int b = 0; b < 2; ++b) {
        w.fif[b] = c.take<double2>(nf);
        w.fef[b] = c.take<double2>(nf);
    }
    w.tf = carve_tend(c, f->plan, 1);
    if (cl) {
        const size_t nc = (size_t)cl->nnodes * 3 * cl->plan->nspec;
        w.thc = c.take<double2>(nc);
        w.thct = c.take<double2>(nc);
        w.fict = c.take<double2>(nc);
        w.fect = c.take<double2>(nc);
        for (int b = 0; b < 2; ++b) {
            w.fic[b] = c.take<double2>(nc);
            w.fec[b] = c.take<double2>(nc);
        }
        w.tau = c.take<double2>(nc);
        w.tc = carve_tend(c, cl->plan, cl->nnodes - 1 > 1 ? cl->nnodes - 1 : 1);
    }
    if (o && o->residual_check) {
        w.rfi = c.take<double2>(nf);
        w.rfe = c.take<double2>(nf);
        w.tr = carve_tend(c, f->plan, f->nnodes);
        w.partial = c.take<double>((size_t)residual_blocks(f->plan) * f->nnodes);
    }
    return w;
}

// Complex and grid arrays are accessed as 16-byte double2.
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

bool valid_params(const swe_params* p) {
    return p && p->a > 0.0;
}

// Round / split the FP64 tables into the plan's working precision and free
// the FP64 copies.  Synchronous (plan creation).
bool convert_tables(shx_plan* p) {
    const int N = p->N, nb = 2 * (N + 1);
    bool ok = true;
    if (p->prec == SHX_FP32) {
        // the untiled FP32 analysis table only where the tiled one is not held
        ok = dalloc(&p->psyn32, p->table_elems) == hipSuccess &&
             (p->pan4f || dalloc(&p->pan32, p->table_elems) == hipSuccess);
        ok = ok && launch_tables_to_f32(p, 0) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    } else {
        const int NP = p->prec == SHX_SPLIT_BF16_2 ? 2 : 3;
        const int Jhp = (p->Jh + 15) / 16 * 16;
        std::vector<int> ra(nb), ca(nb), cpa(nb), rs(nb), cs(nb), cps(nb);
        std::vector<long long> oa(nb), os(nb);
        long long sa = 0, ss = 0;
        for (int m = 0; m <= N; ++m)
            for (int q = 0; q < 2; ++q) {
                const int b = 2 * m + q, K = kcount(p->nmax, m, q), Kp = (K + 15) / 16 * 16;
                ra[b] = K; ca[b] = p->Jh; cpa[b] = Jhp; oa[b] = sa; sa += (long long)K * Jhp;   // [k][jp]
                rs[b] = p->Jh; cs[b] = K; cps[b] = Kp; os[b] = ss; ss += (long long)p->Jh * Kp;  // [jp][k]
            }
        p->an16_plane = (sa + 15) / 16 * 16;
        p->syn16_plane = (ss + 15) / 16 * 16;
        int* d[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        std::vector<int>* h[6] = {&ra, &ca, &cpa, &rs, &cs, &cps};
        ok = dalloc(&p->an16, NP * p->an16_plane) == hipSuccess &&
             dalloc(&p->syn16, NP * p->syn16_plane) == hipSuccess && dalloc(&p->off_an16, nb) == hipSuccess &&
             dalloc(&p->off_syn16, nb) == hipSuccess;
        for (int i = 0; i < 6 && ok; ++i)
            ok = dalloc(&d[i], nb) == hipSuccess &&
                 hipMemcpy(d[i], h[i]->data(), nb * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(p->off_an16, oa.data(), nb * 8, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(p->off_syn16, os.data(), nb * 8, hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && launch_tables_to_bf16(p, d[0], d[1], d[2], d[3], d[4], d[5], 0) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
        for (int i = 0; i < 6; ++i) (void)hipFree(d[i]);
    }
    (void)hipFree(p->psyn);
    (void)hipFree(p->pan);
    p->psyn = p->pan = nullptr;
    return ok;
}

}  // namespace

// Tape of the states at which F is evaluated during a step (fine and
// coarse, in evaluation order), for the adjoint.
struct Tape {
    double2* f;
    double2* c;
};
size_t tape_fine_states(const sdc_level* fl, const mlsdc_opts* o) {
    return 1 + (size_t)o->niter * o->nsweep_fine * (fl->nnodes - 1);
}
size_t tape_coarse_states(const sdc_level* cl, const mlsdc_opts* o) {
    return cl ? 1 + (size_t)o->niter * (cl->nnodes - 1) * (1 + o->nsweep_coarse) : 0;
}

// One MLSDC step (validated arguments); optionally records the tape.
int step_body(const sdc_level* fl, const sdc_level* cl, const mlsdc_opts* o, double dt, const double2* th_n,
              double2* out, double* status, const StepWS& w, const Tape* tape, hipStream_t st) {
    const shx_plan* pf = fl->plan;
    const int Mf = fl->nnodes - 1;
    const size_t nsf3 = 3 * (size_t)pf->nspec;
    // spread: Theta and F at every fine node equal those of Theta^n
    HIPCHK(hipMemcpyAsync(w.thf, th_n, nsf3 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    int rc = tendency_impl(pf, fl->p, 1, w.thf, w.fif[0], w.fef[0], w.tf, st);
    if (rc) return rc;
    if (tape) HIPCHK(hipMemcpyAsync(tape->f, th_n, nsf3 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    {
        NodeCopies nc{};
        nc.add(w.thf, w.thf, 1, Mf);
        nc.add(w.fif[0], w.fif[0], 1, Mf);
        nc.add(w.fef[0], w.fef[0], 1, Mf);
        nc.add(w.fif[0], w.fif[1], 0, 0);
        nc.add(w.fef[0], w.fef[1], 0, 0);
        HIPCHK(launch_node_copies(nc, (long long)nsf3, st));
    }
    int fcur = 0;                                        // fine F buffer holding the current iterate
    Mat9x9 Pcf{}, Pfc{}, PQ{}, Qc{};
    int Mc = 0;
    size_t nsc3 = 0;
    const shx_plan* pc = cl ? cl->plan : nullptr;
    if (cl) {
        Mc = cl->nnodes - 1;
        nsc3 = 3 * (size_t)pc->nspec;
        double a[81], b[81];
        if (shx_host_transfer(fl->kind, fl->nnodes, cl->nnodes, a)) return SHX_EINVAL;   // [nc][nf]
        if (shx_host_transfer(fl->kind, cl->nnodes, fl->nnodes, b)) return SHX_EINVAL;   // [nf][nc]
        Pcf = to_mat(a, cl->nnodes * fl->nnodes);
        Pfc = to_mat(b, fl->nnodes * cl->nnodes);
        // Pi^c_f Q_f  [nc][nf]
        for (int i = 0; i < cl->nnodes; ++i)
            for (int j = 0; j < fl->nnodes; ++j) {
                double sum = 0.0;
                for (int k = 0; k < fl->nnodes; ++k) sum += a[i * fl->nnodes + k] * fl->Q[k * fl->nnodes + j];
                PQ.a[i * fl->nnodes + j] = sum;
            }
        Qc = to_mat(cl->Q, cl->nnodes * cl->nnodes);
        // coarse node 0: restricted initial value and its F, once per step
        Mat9x9 e0{};
        e0.a[0] = 1.0;
        HIPCHK(launch_restrict(pf, pc, e0, 1, 0, 1, th_n, w.thc, w.thct, st));
        rc = tendency_impl(pc, cl->p, 1, w.thct, w.fict, w.fect, w.tc, st);
        if (rc) return rc;
        if (tape) HIPCHK(hipMemcpyAsync(tape->c, w.thct, nsc3 * sizeof(double2), hipMemcpyDeviceToDevice, st));
        NodeCopies nc{};
        for (int b2 = 0; b2 < 2; ++b2) {
            nc.add(w.fict, w.fic[b2], 0, 0);
            nc.add(w.fect, w.fec[b2], 0, 0);
        }
        HIPCHK(launch_node_copies(nc, (long long)nsc3, st));
    }
    for (int k = 0; k < o->niter; ++k) {
        // A) fine sweep(s), old -> new buffers
        for (int s2 = 0; s2 < o->nsweep_fine; ++s2) {
            double2* rec = tape ? tape->f + (1 + (size_t)(k * o->nsweep_fine + s2) * Mf) * nsf3 : nullptr;
            // consecutive sweeps: the F of the last node is formed by the next sweep's first update
            rc = sweep_impl(fl, dt, w.thf, w.fif[fcur], w.fef[fcur], w.fif[1 - fcur], w.fef[1 - fcur], nullptr,
                            w.tf, st, rec, s2 == o->nsweep_fine - 1, s2 > 0);
            if (rc) return rc;
            fcur = 1 - fcur;
        }
        if (!cl) continue;
        // B) restrict nodes 1..Mc (kept twice: iterate and saved copy), evaluate
        HIPCHK(launch_restrict(pf, pc, Pcf, fl->nnodes, 1, cl->nnodes, w.thf, w.thc, w.thct, st));
        rc = tendency_impl(pc, cl->p, Mc, w.thct + nsc3, w.fict + nsc3, w.fect + nsc3, w.tc, st);
        if (rc) return rc;
        const size_t cbase = 1 + (size_t)k * (Mc + o->nsweep_coarse * Mc);
        if (tape)
            HIPCHK(hipMemcpyAsync(tape->c + cbase * nsc3, w.thct + nsc3, Mc * nsc3 * sizeof(double2),
                                  hipMemcpyDeviceToDevice, st));
        // C) FAS correction and coarse sweep(s): the first reads the saved F
        HIPCHK(launch_fas_tau(pf, pc, PQ, Qc, fl->nnodes, cl->nnodes, dt, w.fif[fcur], w.fef[fcur], w.fict, w.fect,
                              w.tau, st));
        const double2 *ci = w.fict, *ce = w.fect;
        for (int s2 = 0; s2 < o->nsweep_coarse; ++s2) {
            double2* rec = tape ? tape->c + (cbase + Mc + (size_t)s2 * Mc) * nsc3 : nullptr;
            rc = sweep_impl(cl, dt, w.thc, ci, ce, w.fic[s2 & 1], w.fec[s2 & 1], w.tau, w.tc, st, rec,
                            s2 == o->nsweep_coarse - 1, s2 > 0);
            if (rc) return rc;
            ci = w.fic[s2 & 1];
            ce = w.fec[s2 & 1];
        }
        // D) interpolate the coarse corrections of Theta, F_I, F_E
        HIPCHK(launch_interp(pf, pc, Pfc, fl->nnodes, cl->nnodes, w.thc, w.thct, ci, w.fict, ce, w.fect, w.thf,
                             w.fif[fcur], w.fef[fcur], st));
    }
    HIPCHK(hipMemcpyAsync(out, w.thf + Mf * nsf3, nsf3 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    if (status) {
        const int nblk = residual_blocks(pf);
        if (o->residual_check) {
            rc = tendency_impl(pf, fl->p, fl->nnodes, w.thf, w.rfi, w.rfe, w.tr, st);
            if (rc) return rc;
            HIPCHK(launch_residual(pf, to_mat(fl->Q, fl->nnodes * fl->nnodes), Mf, dt, w.thf, w.rfi, w.rfe,
                                   w.partial, nblk, st));
        }
        HIPCHK(launch_status(pf, w.partial, nblk, Mf, out, status, o->residual_check, st));
    }
    return SHX_OK;
}

namespace {

// ---------------------------------------------------- multi-level V-cycle
// Per-level buffers of mlsdc_step_multi.  Level 0 (finest): th, fi[2],
// fe[2] and a one-state tendency workspace, as the fine level of step_body.
// Level l >= 1: th (iterate), tht / fit / fet (the restriction and its F,
// kept for the correction), fi[2] / fe[2] (sweep outputs), tau, tmp (the
// restricted tau of level l-1) and an M-state tendency workspace.
struct LevelWS {
    double2 *th, *tht, *fit, *fet, *fi[2], *fe[2], *tau, *tmp;
    TendWS t;
};
LevelWS carve_level(Carve& c, const sdc_level* lv, bool finest) {
    LevelWS w{};
    const size_t n = (size_t)lv->nnodes * 3 * lv->plan->nspec;
    w.th = c.take<double2>(n);
    for (int b = 0; b < 2; ++b) {
        w.fi[b] = c.take<double2>(n);
        w.fe[b] = c.take<double2>(n);
    }
    if (finest) {
        w.t = carve_tend(c, lv->plan, 1);
        return w;
    }
    w.tht = c.take<double2>(n);
    w.fit = c.take<double2>(n);
    w.fet = c.take<double2>(n);
    w.tau = c.take<double2>(n);
    w.tmp = c.take<double2>(n);
    w.t = carve_tend(c, lv->plan, lv->nnodes - 1 > 1 ? lv->nnodes - 1 : 1);
    return w;
}

bool valid_levels(const sdc_level* const* lv, int L) {
    if (!lv || L < 1 || L > SHX_MAX_LEVELS) return false;
    for (int l = 0; l < L; ++l) {
        if (!lv[l]) return false;
        if (l > 0 && (lv[l]->kind != lv[0]->kind || lv[l]->plan->N > lv[l - 1]->plan->N ||
                      lv[l]->nnodes > lv[l - 1]->nnodes))
            return false;
    }
    return true;
}

// One step of the V-cycle over L levels (validated arguments); with L = 2
// the same launches as step_body without tape and status.
int step_multi_body(const sdc_level* const* lv, int L, int niter, const int* ns, double dt, const double2* th_n,
                    double2* out, LevelWS* w, hipStream_t st) {
    const shx_plan* p0 = lv[0]->plan;
    const int M0 = lv[0]->nnodes - 1;
    size_t n3[SHX_MAX_LEVELS];
    for (int l = 0; l < L; ++l) n3[l] = 3 * (size_t)lv[l]->plan->nspec;
    // spread on the finest level
    HIPCHK(hipMemcpyAsync(w[0].th, th_n, n3[0] * sizeof(double2), hipMemcpyDeviceToDevice, st));
    int rc = tendency_impl(p0, lv[0]->p, 1, w[0].th, w[0].fi[0], w[0].fe[0], w[0].t, st);
    if (rc) return rc;
    {
        NodeCopies nc{};
        nc.add(w[0].th, w[0].th, 1, M0);
        nc.add(w[0].fi[0], w[0].fi[0], 1, M0);
        nc.add(w[0].fe[0], w[0].fe[0], 1, M0);
        nc.add(w[0].fi[0], w[0].fi[1], 0, 0);
        nc.add(w[0].fe[0], w[0].fe[1], 0, 0);
        HIPCHK(launch_node_copies(nc, (long long)n3[0], st));
    }
    // transfer matrices of each pair (l-1, l) and node 0 of the coarser levels
    Mat9x9 Pdn[SHX_MAX_LEVELS]{}, Pup[SHX_MAX_LEVELS]{}, PQ[SHX_MAX_LEVELS]{}, Qc[SHX_MAX_LEVELS]{};
    for (int l = 1; l < L; ++l) {
        const int nf = lv[l - 1]->nnodes, nc = lv[l]->nnodes;
        double a[81], b[81];
        if (shx_host_transfer(lv[0]->kind, nf, nc, a)) return SHX_EINVAL;   // [nc][nf]
        if (shx_host_transfer(lv[0]->kind, nc, nf, b)) return SHX_EINVAL;   // [nf][nc]
        Pdn[l] = to_mat(a, nc * nf);
        Pup[l] = to_mat(b, nf * nc);
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nf; ++j) {
                double sum = 0.0;
                for (int k = 0; k < nf; ++k) sum += a[i * nf + k] * lv[l - 1]->Q[k * nf + j];
                PQ[l].a[i * nf + j] = sum;
            }
        Qc[l] = to_mat(lv[l]->Q, nc * nc);
        Mat9x9 e0{};
        e0.a[0] = 1.0;
        HIPCHK(launch_restrict(p0, lv[l]->plan, e0, 1, 0, 1, th_n, w[l].th, w[l].tht, st));
        rc = tendency_impl(lv[l]->plan, lv[l]->p, 1, w[l].tht, w[l].fit, w[l].fet, w[l].t, st);
        if (rc) return rc;
        NodeCopies nc0{};
        for (int b2 = 0; b2 < 2; ++b2) {
            nc0.add(w[l].fit, w[l].fi[b2], 0, 0);
            nc0.add(w[l].fet, w[l].fe[b2], 0, 0);
        }
        HIPCHK(launch_node_copies(nc0, (long long)n3[l], st));
    }
    int fcur = 0;
    for (int k = 0; k < niter; ++k) {
        for (int s2 = 0; s2 < ns[0]; ++s2) {
            rc = sweep_impl(lv[0], dt, w[0].th, w[0].fi[fcur], w[0].fe[fcur], w[0].fi[1 - fcur], w[0].fe[1 - fcur],
                            nullptr, w[0].t, st, nullptr, s2 == ns[0] - 1, s2 > 0);
            if (rc) return rc;
            fcur = 1 - fcur;
        }
        double2 *ci[SHX_MAX_LEVELS], *ce[SHX_MAX_LEVELS];   // current F of each level
        ci[0] = w[0].fi[fcur];
        ce[0] = w[0].fe[fcur];
        for (int l = 1; l < L; ++l) {                     // down: restrict, FAS, sweep
            const shx_plan *pf = lv[l - 1]->plan, *pc = lv[l]->plan;
            const int nf = lv[l - 1]->nnodes, nc = lv[l]->nnodes, Mc = nc - 1;
            HIPCHK(launch_restrict(pf, pc, Pdn[l], nf, 1, nc, w[l - 1].th, w[l].th, w[l].tht, st));
            rc = tendency_impl(pc, lv[l]->p, Mc, w[l].tht + n3[l], w[l].fit + n3[l], w[l].fet + n3[l], w[l].t, st);
            if (rc) return rc;
            HIPCHK(launch_fas_tau(pf, pc, PQ[l], Qc[l], nf, nc, dt, ci[l - 1], ce[l - 1], w[l].fit, w[l].fet,
                                  w[l].tau, st));
            if (l >= 2) {                                 // + the restricted tau of level l-1
                HIPCHK(launch_restrict(pf, pc, Pdn[l], nf, 0, nc, w[l - 1].tau, w[l].tmp, nullptr, st));
                HIPCHK(launch_add(w[l].tmp, w[l].tau, (long long)nc * (long long)n3[l], st));
            }
            const double2 *fi_old = w[l].fit, *fe_old = w[l].fet;
            for (int s2 = 0; s2 < ns[l]; ++s2) {
                rc = sweep_impl(lv[l], dt, w[l].th, fi_old, fe_old, w[l].fi[s2 & 1], w[l].fe[s2 & 1], w[l].tau, w[l].t,
                                st, nullptr, s2 == ns[l] - 1, s2 > 0);
                if (rc) return rc;
                fi_old = w[l].fi[s2 & 1];
                fe_old = w[l].fe[s2 & 1];
            }
            ci[l] = w[l].fi[(ns[l] - 1) & 1];
            ce[l] = w[l].fe[(ns[l] - 1) & 1];
        }
        for (int l = L - 1; l >= 1; --l)                  // up: corrections of level l into level l-1
            HIPCHK(launch_interp(lv[l - 1]->plan, lv[l]->plan, Pup[l], lv[l - 1]->nnodes, lv[l]->nnodes, w[l].th,
                                 w[l].tht, ci[l], w[l].fit, ce[l], w[l].fet, w[l - 1].th, ci[l - 1], ce[l - 1], st));
    }
    HIPCHK(hipMemcpyAsync(out, w[0].th + M0 * n3[0], n3[0] * sizeof(double2), hipMemcpyDeviceToDevice, st));
    return SHX_OK;
}

}  // namespace

namespace {

// ------------------------------------------------------------------ adjoint
// Workspace of the tendency adjoint for S states.
struct TendAdjWS {
    double2 *FIs, *FIl, *Ga, *lam4;
    double* grid;                   // grid rows in HBM for row lengths beyond the LDS kernel
};
TendAdjWS carve_tadj(Carve& c, const shx_plan* pl, int S) {
    TendAdjWS t;
    const size_t fj = (size_t)S * pl->J * (pl->N + 1);
    t.FIs = c.take<double2>(fj * 4);
    t.FIl = c.take<double2>(fj * 5);
    t.Ga = c.take<double2>(fj * 4);
    t.lam4 = c.take<double2>((size_t)S * pl->nspec_e * 4);
    const size_t gd = adj_grid_doubles(pl, S);
    t.grid = gd ? c.take<double>(gd) : nullptr;
    return t;
}

// lstate += (dF_I/dTheta)^T lfi + (dF_E/dTheta)^T lfe, linearised at `state`.
int tendency_adj_impl(const shx_plan* pl, const swe_params& p, int S, const double2* state, const double2* lfi,
                      const double2* lfe, double2* lstate, const TendAdjWS& t, hipStream_t st) {
    if (lfe) {
        HIPCHK(launch_leg_syn_swe(pl, p.a, state, t.FIs, S, st));
        HIPCHK(launch_leg_syn_swe_adj(pl, p.a, lfe, t.FIl, S, st));
        HIPCHK(launch_swe_grid_adj(pl, t.FIs, t.FIl, t.Ga, S, p.omega, t.grid, st));
        HIPCHK(launch_leg_an(pl, t.Ga, t.lam4, 4, S, pl->nmax, st));
    }
    HIPCHK(launch_prep_adj(pl, p, t.lam4, lfi, lstate, S, lfe != nullptr, st));
    return SHX_OK;
}

// Transpose of sweep_impl.  states: the M states at which the sweep evaluated
// F (nodes 1..M).  In: lth (adjoint of the output Theta; node 0 accumulates),
// lfi_out/lfe_out (adjoint of the output F; used as work).  Out: lfi_in/lfe_in
// (adjoint of the input F; must be zero on entry), ltau accumulated.
int sweep_adj_impl(const sdc_level* lv, double dt, const double2* states, double2* lth, double2* lfi_out,
                   double2* lfe_out, double2* lfi_in, double2* lfe_in, double2* ltau, const TendAdjWS& t,
                   hipStream_t st) {
    const shx_plan* pl = lv->plan;
    const int M = lv->nnodes - 1, n1 = lv->nnodes;
    const size_t ns3 = 3 * (size_t)pl->nspec;
    {   // node 0 passes through
        ArrayList a{};
        a.add(lfi_in, lfi_out);
        a.add(lfe_in, lfe_out);
        HIPCHK(launch_add_n(a, (long long)ns3, st));
    }
    for (int m = M - 1; m >= 0; --m) {
        const size_t o = (size_t)(m + 1) * ns3;
        int rc = tendency_adj_impl(pl, lv->p, 1, states + (size_t)m * ns3, lfi_out + o, lfe_out + o, lth + o, t, st);
        if (rc) return rc;
        NodeWeights wt;
        for (int j = 0; j < 9; ++j) {
            const bool in = j < n1;
            wt.q[j] = in ? dt * lv->Q[(m + 1) * n1 + j] : 0.0;
            wt.qe[j] = in ? dt * lv->QE[(m + 1) * n1 + j] : 0.0;
            wt.qd[j] = in ? dt * lv->QD[(m + 1) * n1 + j] : 0.0;
        }
        const double h = dt * lv->QD[(m + 1) * n1 + (m + 1)];
        HIPCHK(launch_sdc_node_adj(pl, lv->p, m, M, wt, h, lth, lfi_out, lfe_out, lfi_in, lfe_in, ltau, st));
    }
    return SHX_OK;
}

// Transfer matrices of a level pair: Pcf [nc][nf], Pfc [nf][nc], PQ = Pcf Q_f, Qc.
int level_pair_matrices(const sdc_level* fl, const sdc_level* cl, Mat9x9& Pcf, Mat9x9& Pfc, Mat9x9& PQ,
                        Mat9x9& Qc) {
    double a[81], b[81];
    if (shx_host_transfer(fl->kind, fl->nnodes, cl->nnodes, a)) return SHX_EINVAL;
    if (shx_host_transfer(fl->kind, cl->nnodes, fl->nnodes, b)) return SHX_EINVAL;
    Pcf = to_mat(a, cl->nnodes * fl->nnodes);
    Pfc = to_mat(b, fl->nnodes * cl->nnodes);
    std::memset(&PQ, 0, sizeof(PQ));
    for (int i = 0; i < cl->nnodes; ++i)
        for (int j = 0; j < fl->nnodes; ++j) {
            double sum = 0.0;
            for (int k = 0; k < fl->nnodes; ++k) sum += a[i * fl->nnodes + k] * fl->Q[k * fl->nnodes + j];
            PQ.a[i * fl->nnodes + j] = sum;
        }
    Qc = to_mat(cl->Q, cl->nnodes * cl->nnodes);
    return SHX_OK;
}

struct StepAdjWS {
    StepWS fw;
    Tape tape;
    double2 *lthf, *lff[2][2];                 // fine: Theta, F buffers [b][fi/fe], [Mf+1][3][nsf]
    double2 *lthc, *lthct, *lfict, *lfect, *lfc[2][2], *ltau;   // coarse [Mc+1][3][nsc]
    double2 *lthc0, *lfic0, *lfec0;           // coarse node 0 accumulators [3][nsc]
    double2 *lsfi, *lsfe;                     // fine node sums [3][nsf]
    TendAdjWS tf, tc;
};
StepAdjWS carve_step_adj(Carve& c, const sdc_level* f, const sdc_level* cl, const mlsdc_opts* o) {
    StepAdjWS w{};
    mlsdc_opts fo = *o;
    fo.residual_check = 0;
    w.fw = carve_step(c, f, cl, &fo);
    const size_t nf3 = 3 * (size_t)f->plan->nspec, nf = (size_t)f->nnodes * nf3;
    w.tape.f = c.take<double2>(tape_fine_states(f, o) * nf3);
    w.lthf = c.take<double2>(nf);
    for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 2; ++q) w.lff[b][q] = c.take<double2>(nf);
    w.lsfi = c.take<double2>(nf3);
    w.lsfe = c.take<double2>(nf3);
    w.tf = carve_tadj(c, f->plan, 1);
    w.tape.c = nullptr;
    if (cl) {
        const size_t nc3 = 3 * (size_t)cl->plan->nspec, nc = (size_t)cl->nnodes * nc3;
        w.tape.c = c.take<double2>(tape_coarse_states(cl, o) * nc3);
        w.lthc = c.take<double2>(nc);
        w.lthct = c.take<double2>(nc);
        w.lfict = c.take<double2>(nc);
        w.lfect = c.take<double2>(nc);
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) w.lfc[b][q] = c.take<double2>(nc);
        w.ltau = c.take<double2>(nc);
        w.lthc0 = c.take<double2>(nc3);
        w.lfic0 = c.take<double2>(nc3);
        w.lfec0 = c.take<double2>(nc3);
        w.tc = carve_tadj(c, cl->plan, cl->nnodes - 1 > 1 ? cl->nnodes - 1 : 1);
    }
    return w;
}

}  // namespace

// ------------------------------------------------ allocation-free step
// The workspace of mlsdc_step_noalloc: one array per device, held from the
// first use of the library on that device until the process ends.  In host
// code the name `scratch` is only a stand-in for the device symbol; its
// device address (different on every device) is looked up once per device
// with hipGetSymbolAddress and cached, and only that address is passed on.
namespace {
static __device__ __align__(256) unsigned char scratch[SHX_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEV = 64;
void* g_scratch_ptr[SCRATCH_MAX_DEV] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on device dev (looked up with dev current),
// or nullptr if the lookup fails.
void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
    return ptr;
}
}  // namespace

extern "C" {

size_t shx_nspec(int ntrunc) { return ntrunc < 0 ? 0 : (size_t)nspec_of(ntrunc); }

int shx_kernel_timer_start(int kclass, int capacity) {
    if (kclass < 0 || kclass > SHX_KC_SDC_NODE || capacity < 1) return SHX_EINVAL;
    shx_kernel_timer_stop(nullptr, nullptr);
    g_timer.ev0.resize(capacity);
    g_timer.ev1.resize(capacity);
    for (int i = 0; i < capacity; ++i) {
        if (hipEventCreate(&g_timer.ev0[i]) != hipSuccess || hipEventCreate(&g_timer.ev1[i]) != hipSuccess) {
            g_timer.cap = i;
            shx_kernel_timer_stop(nullptr, nullptr);
            return SHX_EHIP;
        }
    }
    g_timer.cap = capacity;
    g_timer.n = 0;
    g_timer.kclass = kclass;
    return SHX_OK;
}

int shx_kernel_timer_stop(float* ms, int* count) {
    int rc = SHX_OK;
    if (count) *count = g_timer.n;
    for (int i = 0; i < g_timer.n && ms; ++i) {
        if (hipEventSynchronize(g_timer.ev1[i]) != hipSuccess ||
            hipEventElapsedTime(&ms[i], g_timer.ev0[i], g_timer.ev1[i]) != hipSuccess)
            rc = SHX_EHIP;
    }
    for (int i = 0; i < g_timer.cap; ++i) {
        (void)hipEventDestroy(g_timer.ev0[i]);
        (void)hipEventDestroy(g_timer.ev1[i]);
    }
    g_timer.ev0.clear();
    g_timer.ev1.clear();
    g_timer.kclass = -1;
    g_timer.cap = g_timer.n = 0;
    return rc;
}

const char* shx_strerror(int s) {
    switch (s) {
        case SHX_OK: return "ok";
        case SHX_EINVAL: return "invalid argument";
        case SHX_ESHAPE: return "grid too small for the truncation";
        case SHX_EUNSUPPORTED: return "unsupported size or option";
        case SHX_EWORKSPACE: return "workspace missing or too small";
        case SHX_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

int shx_plan_create(int N, int J, int I, int prec, int table_mode, shx_plan** out) {
    if (!out || N < 1 || J < 2 || I < 2) return SHX_EINVAL;
    *out = nullptr;
    if (table_mode != SHX_TABLE_HBM && table_mode != SHX_TABLE_ONTHEFLY) return SHX_EINVAL;
    if (prec < SHX_FP64 || prec > SHX_SPLIT_BF16_3) return SHX_EUNSUPPORTED;
    if ((J & 1) || I <= 2 * N || J <= N) return SHX_ESHAPE;
    if (!fft_length_supported(I)) return SHX_EUNSUPPORTED;
    shx_plan* p = new (std::nothrow) shx_plan();
    if (!p) return SHX_EINVAL;
    p->N = N;
    p->J = J;
    p->I = I;
    p->prec = prec;
    p->tmode = table_mode;
    p->nmax = N + 1;
    p->Jh = J / 2;
    p->nspec = nspec_of(N);
    p->nspec_e = nspec_ext_of(N);
    if (hipGetDevice(&p->dev) != hipSuccess) { delete p; return SHX_EHIP; }
    p->h_mu.resize(J);
    p->h_sint.resize(J);
    p->h_cos2.resize(J);
    p->h_w.resize(J);
    if (shx_host_gauss(J, p->h_mu.data(), p->h_sint.data(), p->h_cos2.data(), p->h_w.data())) {
        delete p;
        return SHX_EINVAL;
    }
    std::vector<double> twr(I), twi(I);
    shx_host_twiddles(I, twr.data(), twi.data());
    std::vector<double2> tw(I);
    for (int t = 0; t < I; ++t) tw[t] = make_double2(twr[t], twi[t]);
    // table offsets per (m, p)
    p->h_off.resize(2 * (N + 1));
    long long acc = 0;
    for (int m = 0; m <= N; ++m)
        for (int q = 0; q < 2; ++q) {
            p->h_off[2 * m + q] = acc;
            acc += (long long)kcount(p->nmax, m, q) * p->Jh;
        }
    p->table_elems = acc;
    std::vector<long long> ckoff(N + 1);
    long long ck_elems = 0;
    for (int m = 0; m <= N; ++m) {
        ckoff[m] = ck_elems;
        ck_elems += 4LL * seg_rounds(p->nmax - m + 1) * p->Jh;
    }
    // analysis blocks: per XCD x the (m, g) of the orders m = x mod 8, in order
    std::vector<std::vector<int>> xl(8);
    for (int m = 0; m <= N; ++m)
        for (int g = 0; g < 4 * seg_rounds(p->nmax - m + 1); ++g) {
            xl[m % 8].push_back(m);
            xl[m % 8].push_back(g);
        }
    size_t nslot = 0;
    for (auto& v : xl) nslot = v.size() / 2 > nslot ? v.size() / 2 : nslot;
    std::vector<int> anblk(16 * nslot, -1);
    for (size_t t = 0; t < nslot; ++t)
        for (int x = 0; x < 8; ++x)
            if (2 * t < xl[x].size()) {
                anblk[2 * (8 * t + x)] = xl[x][2 * t];
                anblk[2 * (8 * t + x) + 1] = xl[x][2 * t + 1];
            }
    p->an_nblk = (int)(8 * nslot);
    // table-analysis blocks: per XCD x the (m, p, tile) of the orders m = x mod 8
    std::vector<std::vector<int>> tl(8);
    for (int m = 0; m <= N; ++m)
        for (int q = 0; q < 2; ++q)
            for (int t = 0; t * 64 < kcount(p->nmax, m, q); ++t) {
                tl[m % 8].push_back(2 * m + q);
                tl[m % 8].push_back(t);
            }
    size_t tslot = 0;
    for (auto& v : tl) tslot = v.size() / 2 > tslot ? v.size() / 2 : tslot;
    std::vector<int> tblk(16 * tslot, -1);
    for (size_t t = 0; t < tslot; ++t)
        for (int x = 0; x < 8; ++x)
            if (2 * t < tl[x].size()) {
                tblk[2 * (8 * t + x)] = tl[x][2 * t];
                tblk[2 * (8 * t + x) + 1] = tl[x][2 * t + 1];
            }
    p->tb_nblk = (int)(8 * tslot);
    // degree factors of the tendency rows (eps_nm as on the device: correctly
    // rounded FP64 sqrt and division)
    std::vector<double2> pf(p->nspec_e);
    std::vector<double> ninv(N + 3), nn1(N + 3);
    for (int m = 0; m <= N; ++m)
        for (int n = m; n <= N + 1; ++n)
            pf[ext_idx(N, m, n)] = make_double2((n - 1.0) * eps_nm(n, m), (n + 2.0) * eps_nm(n + 1, m));
    for (int n = 0; n <= N + 2; ++n) {
        nn1[n] = n * (n + 1.0);
        ninv[n] = n > 0 ? -1.0 / nn1[n] : 0.0;
    }
    std::vector<int> ord(p->nspec), deg(p->nspec), orde(p->nspec_e), dege(p->nspec_e);
    for (int m = 0; m <= N; ++m) {
        for (int n = m; n <= N; ++n) {
            ord[spec_idx(N, m, n)] = m;
            deg[spec_idx(N, m, n)] = n;
        }
        for (int n = m; n <= N + 1; ++n) {
            orde[ext_idx(N, m, n)] = m;
            dege[ext_idx(N, m, n)] = n;
        }
    }
    bool ok = dalloc(&p->mu, J) == hipSuccess && dalloc(&p->sint, J) == hipSuccess &&
              dalloc(&p->cos2, J) == hipSuccess && dalloc(&p->w, J) == hipSuccess &&
              dalloc(&p->tw, I) == hipSuccess &&
              (table_mode == SHX_TABLE_ONTHEFLY ||
               (dalloc(&p->psyn, acc) == hipSuccess && dalloc(&p->pan, acc) == hipSuccess)) &&
              dalloc(&p->off, p->h_off.size()) == hipSuccess &&
              dalloc(&p->ord, p->nspec) == hipSuccess && dalloc(&p->deg, p->nspec) == hipSuccess &&
              dalloc(&p->ord_e, p->nspec_e) == hipSuccess && dalloc(&p->deg_e, p->nspec_e) == hipSuccess &&
              dalloc(&p->ck, ck_elems) == hipSuccess && dalloc(&p->ckoff, N + 1) == hipSuccess &&
              dalloc(&p->rc, p->nspec_e) == hipSuccess && dalloc(&p->anblk, anblk.size()) == hipSuccess &&
              dalloc(&p->rq, p->nspec_e) == hipSuccess && dalloc(&p->cs, p->nspec_e) == hipSuccess &&
              dalloc(&p->pf, p->nspec_e) == hipSuccess && dalloc(&p->ninv, N + 3) == hipSuccess &&
              dalloc(&p->nn1, N + 3) == hipSuccess;
    ok = ok && hipMemcpy(p->pf, pf.data(), pf.size() * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->ninv, ninv.data(), (N + 3) * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->nn1, nn1.data(), (N + 3) * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->anblk, anblk.data(), anblk.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->ckoff, ckoff.data(), (N + 1) * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(p->ck, 0, ck_elems * sizeof(double2)) == hipSuccess;
    ok = ok && hipMemcpy(p->mu, p->h_mu.data(), J * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->sint, p->h_sint.data(), J * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->cos2, p->h_cos2.data(), J * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->w, p->h_w.data(), J * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->tw, tw.data(), I * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->off, p->h_off.data(), p->h_off.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->ord, ord.data(), ord.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->deg, deg.data(), deg.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->ord_e, orde.data(), orde.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(p->deg_e, dege.data(), dege.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && launch_plm_table(p, 0) == hipSuccess;
    if (ok && table_mode == SHX_TABLE_HBM &&
        ((prec == SHX_FP64 && p->Jh <= AN_TAB_JH) || (prec == SHX_FP32 && p->Jh <= AN_TAB_JH_F32))) {
        // the analysis table in the layout of the matrix-core table analysis
        // (FP64, or rounded to FP32 for SHX_FP32 plans)
        const int ngrp = (p->Jh + 3) / 4;
        std::vector<long long> off4(2 * (N + 1));
        long long tot = 0, mx = 0;
        for (int mp = 0; mp < 2 * (N + 1); ++mp) {
            // whole tiles of 64 values per latitude group, the last tile
            // 4 x its rows per group
            const int K = kcount(p->nmax, mp >> 1, mp & 1), nt = (K + 15) / 16;
            const long long sz = K > 0 ? ((long long)(nt - 1) * 64 + 4 * (K - 16 * (nt - 1))) * ngrp : 0;
            off4[mp] = tot;
            tot += sz;
            const long long padded = (long long)nt * ngrp * 64;
            mx = padded > mx ? padded : mx;
        }
        p->an_kt = (kcount(p->nmax, 0, 0) + 15) / 16;   // tiles of the largest block (m = 0, p = 0)
        ok = (prec == SHX_FP64 ? dalloc(&p->pan4, tot) : dalloc(&p->pan4f, tot)) == hipSuccess &&
             dalloc(&p->off4, off4.size()) == hipSuccess &&
             dalloc(&p->an_c0, (size_t)2 * (N + 1) * p->an_kt) == hipSuccess &&
             hipMemcpy(p->off4, off4.data(), off4.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
             launch_an_tab4(p, mx, 0) == hipSuccess && launch_an_polar(p, 0) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
        // block list with the first summed latitude group of each of the
        // block's four tiles (a byte each) and their minimum
        p->h_an_c0.assign((size_t)2 * (N + 1) * p->an_kt, 0);
        ok = ok && hipMemcpy(p->h_an_c0.data(), p->an_c0, p->h_an_c0.size() * sizeof(int),
                             hipMemcpyDeviceToHost) == hipSuccess;
        const int B = an_batch(p->Jh);
        for (int& c : p->h_an_c0) {                     // whole batches of loads from the first summed group
            const int run = B * ((ngrp - c + B - 1) / B);
            c = ngrp - run > 0 ? ngrp - run : 0;
        }
        (void)hipFree(p->an_c0);
        p->an_c0 = nullptr;
        std::vector<int> tb4(4 * (size_t)p->tb_nblk, -1);
        for (int b = 0; ok && b < p->tb_nblk; ++b) {
            const int mp = tblk[2 * b], tx = tblk[2 * b + 1];
            if (mp < 0) continue;
            const int K = kcount(p->nmax, mp >> 1, mp & 1);
            unsigned packed = 0;
            int cmin = ngrp;
            for (int w = 0; w < 4; ++w) {
                const int kt = 4 * tx + w;
                const int c = (16 * kt < K) ? p->h_an_c0[(size_t)mp * p->an_kt + kt] : ngrp;
                packed |= (unsigned)c << (8 * w);
                cmin = c < cmin ? c : cmin;
            }
            tb4[4 * b] = mp;
            tb4[4 * b + 1] = tx;
            tb4[4 * b + 2] = (int)packed;
            tb4[4 * b + 3] = cmin;
        }
        ok = ok && dalloc(&p->tblk, tb4.size()) == hipSuccess &&
             hipMemcpy(p->tblk, tb4.data(), tb4.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        if (ok && prec == SHX_FP64) {                   // the [m][p][jp][k] layout has no other reader here
            (void)hipFree(p->pan);
            p->pan = nullptr;
        }
    }
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (ok && prec != SHX_FP64 && table_mode == SHX_TABLE_HBM) ok = convert_tables(p);
    if (!ok) {
        plan_free(p);
        return SHX_EHIP;
    }
    *out = p;
    return SHX_OK;
}

void shx_plan_destroy(shx_plan* plan) { plan_free(plan); }

int shx_plan_latitudes(const shx_plan* pl, double* mu, double* st, double* w) {
    if (!pl) return SHX_EINVAL;
    for (int j = 0; j < pl->J; ++j) {
        if (mu) mu[j] = pl->h_mu[j];
        if (st) st[j] = pl->h_sint[j];
        if (w) w[j] = pl->h_w[j];
    }
    return SHX_OK;
}

int shx_plan_analysis_terms(const shx_plan* pl, int nmax, long long* terms, long long* fourier_pairs) {
    if (!pl || !terms || (nmax != pl->N && nmax != pl->N + 1)) return SHX_EINVAL;
    const std::vector<int>& c0 = pl->h_an_c0;
    long long t = 0, fp = 0;
    for (int m = 0; m <= pl->N; ++m) {
        int first = pl->Jh;                             // first latitude pair read for this order
        for (int p = 0; p < 2; ++p) {
            const int mp = 2 * m + p, K = kcount(nmax, m, p);
            for (int kt = 0; 16 * kt < K; ++kt) {
                const int rows = K - 16 * kt < 16 ? K - 16 * kt : 16;
                int j0 = (pl->pan4 || pl->pan4f) ? 4 * c0[(size_t)mp * pl->an_kt + kt] : 0;
                j0 = j0 < pl->Jh ? j0 : pl->Jh;
                t += (long long)rows * (pl->Jh - j0);
                first = j0 < first ? j0 : first;
            }
        }
        fp += pl->Jh - first;
    }
    *terms = t;
    if (fourier_pairs) *fourier_pairs = fp;
    return SHX_OK;
}

int shx_plan_legendre(const shx_plan* pl, int m, int n, double* out) {
    if (!pl || !out || m < 0 || m > pl->N || n < m || n > pl->nmax) return SHX_EINVAL;
    const int p = (n - m) & 1, k = (n - m) >> 1;
    const long long o = pl->h_off[2 * m + p] + (long long)k * pl->Jh;   // row k of the [k][jp] layout
    if (pl->tmode == SHX_TABLE_ONTHEFLY) {
        // no table: the row from the recurrence, then the working precision's
        // rounding (FP32) or split (sum of the bf16 pieces) that the contractions use
        double* d = nullptr;
        if (dalloc(&d, pl->Jh) != hipSuccess) return SHX_EHIP;
        const bool ok = launch_plm_one(pl, m, n, d, 0) == hipSuccess &&
                        hipMemcpy(out, d, pl->Jh * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
        (void)hipFree(d);
        if (!ok) return SHX_EHIP;
        for (int j = 0; j < pl->Jh; ++j) out[j] = shx_host_working_value(pl->prec, out[j]);
        return SHX_OK;
    }
    if (pl->prec == SHX_FP64) {
        if (hipMemcpy(out, pl->psyn + o, pl->Jh * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return SHX_EHIP;
    } else if (pl->prec == SHX_FP32) {
        std::vector<float> t(pl->Jh);
        if (hipMemcpy(t.data(), pl->psyn32 + o, pl->Jh * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            return SHX_EHIP;
        for (int j = 0; j < pl->Jh; ++j) out[j] = t[j];
    } else {
        // analysis planes hold [k][jp pad 16] per (m, p): sum of the split planes
        const int NP = pl->prec == SHX_SPLIT_BF16_2 ? 2 : 3;
        const int Jhp = (pl->Jh + 15) / 16 * 16;
        long long o16 = 0;
        for (int b = 0; b < 2 * m + p; ++b) o16 += (long long)kcount(pl->nmax, b / 2, b % 2) * Jhp;
        o16 += (long long)k * Jhp;
        for (int j = 0; j < pl->Jh; ++j) out[j] = 0.0;
        std::vector<unsigned short> t(pl->Jh);
        for (int q = 0; q < NP; ++q) {
            if (hipMemcpy(t.data(), pl->an16 + q * pl->an16_plane + o16, pl->Jh * 2, hipMemcpyDeviceToHost) !=
                hipSuccess)
                return SHX_EHIP;
            for (int j = 0; j < pl->Jh; ++j) {
                const unsigned u = (unsigned)t[j] << 16;
                float f;
                std::memcpy(&f, &u, 4);
                out[j] += f;
            }
        }
    }
    return SHX_OK;
}

size_t shx_workspace_bytes(const shx_plan* pl, int F) {
    if (!pl || F < 1) return 0;
    return align256((size_t)pl->nspec_e * F * sizeof(double2)) +
           align256((size_t)pl->J * (pl->N + 1) * F * sizeof(double2));
}

int sh_inverse(const shx_plan* pl, int F, const double* spec, double* grid, void* ws, size_t wsb,
               shx_stream_t stream) {
    if (!pl || F < 1 || !spec || !grid || !aligned16(spec) || !aligned16(grid)) return SHX_EINVAL;
    if (!ws || wsb < shx_workspace_bytes(pl, F)) return SHX_EWORKSPACE;
    Carve c{static_cast<char*>(ws)};
    double2* cin = c.take<double2>((size_t)pl->nspec_e * F);
    double2* FI = c.take<double2>((size_t)pl->J * (pl->N + 1) * F);
    hipStream_t st = S(stream);
    HIPCHK(launch_spec_to_ext(pl, reinterpret_cast<const double2*>(spec), cin, F, 0, st));
    HIPCHK(timed(SHX_KC_LEGENDRE_SYN, st, [&] { return launch_leg_syn(pl, cin, FI, F, 1, pl->N, st); }));
    HIPCHK(launch_fft_inv(pl, FI, grid, F, 0, st));
    return SHX_OK;
}

int sh_forward(const shx_plan* pl, int F, const double* grid, double* spec, void* ws, size_t wsb,
               shx_stream_t stream) {
    if (!pl || F < 1 || !spec || !grid || !aligned16(spec) || !aligned16(grid)) return SHX_EINVAL;
    if (!ws || wsb < shx_workspace_bytes(pl, F)) return SHX_EWORKSPACE;
    Carve c{static_cast<char*>(ws)};
    double2* cout = c.take<double2>((size_t)pl->nspec_e * F);
    double2* G = c.take<double2>((size_t)pl->J * (pl->N + 1) * F);
    hipStream_t st = S(stream);
    HIPCHK(launch_fft_fwd(pl, grid, G, F, 0, st));
    HIPCHK(timed(SHX_KC_LEGENDRE_AN, st, [&] { return launch_leg_an(pl, G, cout, F, 1, pl->N, st); }));
    HIPCHK(launch_ext_to_spec(pl, cout, reinterpret_cast<double2*>(spec), F, st));
    return SHX_OK;
}

size_t swe_adj_workspace_bytes(const shx_plan* pl, int nstate) {
    if (!pl || nstate < 1) return 0;
    Carve c{nullptr};
    carve_tadj(c, pl, nstate);
    return c.used;
}

int swe_tendency_adj(const shx_plan* pl, const swe_params* prm, int nst, const double* state, const double* lfi,
                     const double* lfe, double* lstate, void* ws, size_t wsb, shx_stream_t stream) {
    if (!pl || !valid_params(prm) || nst < 1 || !state || !lstate || !aligned16(state) || !aligned16(lfi) ||
        !aligned16(lfe) || !aligned16(lstate) || !aligned16(ws))
        return SHX_EINVAL;
    if (!alias_free(pl)) return SHX_ESHAPE;
    if (pl->prec != SHX_FP64 || (lfe && !adjoint_length_supported(pl->I))) return SHX_EUNSUPPORTED;
    if (!ws || wsb < swe_adj_workspace_bytes(pl, nst)) return SHX_EWORKSPACE;
    Carve c{static_cast<char*>(ws)};
    TendAdjWS t = carve_tadj(c, pl, nst);
    return tendency_adj_impl(pl, *prm, nst, reinterpret_cast<const double2*>(state),
                             reinterpret_cast<const double2*>(lfi), reinterpret_cast<const double2*>(lfe),
                             reinterpret_cast<double2*>(lstate), t, S(stream));
}

int imex_solve_adj(const shx_plan* pl, const swe_params* prm, int nst, double h, const double* lam_out,
                   double* lam_rhs, shx_stream_t stream) {
    if (!pl || !valid_params(prm) || nst < 1 || !lam_out || !lam_rhs || !(h >= 0.0) || !aligned16(lam_out) ||
        !aligned16(lam_rhs))
        return SHX_EINVAL;
    HIPCHK(launch_imex_solve_adj(pl, *prm, h, reinterpret_cast<const double2*>(lam_out),
                                 reinterpret_cast<double2*>(lam_rhs), nst, S(stream)));
    return SHX_OK;
}

int sh_inverse_adj(const shx_plan* pl, int F, const double* grid_cot, double* spec_cot, void* ws, size_t wsb,
                   shx_stream_t stream) {
    if (!pl || F < 1 || !grid_cot || !spec_cot || !aligned16(grid_cot) || !aligned16(spec_cot)) return SHX_EINVAL;
    if (pl->prec != SHX_FP64) return SHX_EUNSUPPORTED;
    if (!ws || wsb < shx_workspace_bytes(pl, F)) return SHX_EWORKSPACE;
    Carve c{static_cast<char*>(ws)};
    double2* cout = c.take<double2>((size_t)pl->nspec_e * F);
    double2* G = c.take<double2>((size_t)pl->J * (pl->N + 1) * F);
    hipStream_t st = S(stream);
    HIPCHK(launch_fft_fwd(pl, grid_cot, G, F, 1, st));
    HIPCHK(launch_leg_an(pl, G, cout, F, 1, pl->N, st));
    HIPCHK(launch_ext_to_spec(pl, cout, reinterpret_cast<double2*>(spec_cot), F, st));
    return SHX_OK;
}

int sh_forward_adj(const shx_plan* pl, int F, const double* spec_cot, double* grid_cot, void* ws, size_t wsb,
                   shx_stream_t stream) {
    if (!pl || F < 1 || !grid_cot || !spec_cot || !aligned16(grid_cot) || !aligned16(spec_cot)) return SHX_EINVAL;
    if (pl->prec != SHX_FP64) return SHX_EUNSUPPORTED;
    if (!ws || wsb < shx_workspace_bytes(pl, F)) return SHX_EWORKSPACE;
    Carve c{static_cast<char*>(ws)};
    double2* cin = c.take<double2>((size_t)pl->nspec_e * F);
    double2* FI = c.take<double2>((size_t)pl->J * (pl->N + 1) * F);
    hipStream_t st = S(stream);
    HIPCHK(launch_spec_to_ext(pl, reinterpret_cast<const double2*>(spec_cot), cin, F, 1, st));
    HIPCHK(launch_leg_syn(pl, cin, FI, F, 1, pl->N, st));
    HIPCHK(launch_fft_inv(pl, FI, grid_cot, F, 1, st));
    return SHX_OK;
}

size_t mlsdc_adj_workspace_bytes(const sdc_level* f, const sdc_level* c, const mlsdc_opts* o) {
    if (!f || !o) return 0;
    Carve cv{nullptr};
    carve_step_adj(cv, f, c, o);
    return cv.used;
}

int mlsdc_step_adj(const sdc_level* fl, const sdc_level* cl, const mlsdc_opts* o, double dt, const double* theta_n,
                   const double* lam_np1, double* lam_n, void* ws, size_t wsb, shx_stream_t stream) {
    if (!fl || !o || !theta_n || !lam_np1 || !lam_n || !(dt > 0.0) || o->niter < 0 || o->nsweep_fine < 1 ||
        (cl && o->nsweep_coarse < 1) || !aligned16(theta_n) || !aligned16(lam_np1) || !aligned16(lam_n) ||
        !aligned16(ws) || lam_n == lam_np1 || lam_n == theta_n)
        return SHX_EINVAL;
    if (cl && (cl->kind != fl->kind || cl->plan->N > fl->plan->N || cl->nnodes > fl->nnodes))
        return SHX_EINVAL;
    if (!alias_free(fl->plan) || (cl && !alias_free(cl->plan))) return SHX_ESHAPE;
    if (!adjoint_length_supported(fl->plan->I) || (cl && !adjoint_length_supported(cl->plan->I)) ||
        fl->plan->prec != SHX_FP64 || (cl && cl->plan->prec != SHX_FP64))
        return SHX_EUNSUPPORTED;
    if (!ws || wsb < mlsdc_adj_workspace_bytes(fl, cl, o)) return SHX_EWORKSPACE;
    Carve cv{static_cast<char*>(ws)};
    StepAdjWS w = carve_step_adj(cv, fl, cl, o);
    hipStream_t st = S(stream);
    const shx_plan* pf = fl->plan;
    const int Mf = fl->nnodes - 1, nsf = o->nsweep_fine;
    const size_t nf3 = 3 * (size_t)pf->nspec, nfa = (size_t)fl->nnodes * nf3;
    const double2* th_n = reinterpret_cast<const double2*>(theta_n);
    double2* lout = reinterpret_cast<double2*>(lam_n);
    // 1. forward recompute from the checkpoint, recording the tape (output into lam_n as scratch)
    mlsdc_opts fo = *o;
    fo.residual_check = 0;
    int rc = step_body(fl, cl, &fo, dt, th_n, lout, nullptr, w.fw, &w.tape, st);
    if (rc) return rc;
    // 2. reverse pass
    {
        ArrayList z{};
        z.add(w.lthf);
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) z.add(w.lff[b][q]);
        HIPCHK(launch_zero_n(z, (long long)nfa, st));
    }
    HIPCHK(hipMemcpyAsync(w.lthf + Mf * nf3, lam_np1, nf3 * sizeof(double2), hipMemcpyDeviceToDevice, st));
    const shx_plan* pc = cl ? cl->plan : nullptr;
    int Mc = 0, nsc = 0;
    size_t nc3 = 0, nca = 0;
    Mat9x9 Pcf{}, Pfc{}, PQ{}, Qc{};
    if (cl) {
        Mc = cl->nnodes - 1;
        nsc = o->nsweep_coarse;
        nc3 = 3 * (size_t)pc->nspec;
        nca = (size_t)cl->nnodes * nc3;
        if (level_pair_matrices(fl, cl, Pcf, Pfc, PQ, Qc)) return SHX_EINVAL;
        ArrayList z{};
        z.add(w.lthc0);
        z.add(w.lfic0);
        z.add(w.lfec0);
        HIPCHK(launch_zero_n(z, (long long)nc3, st));
    }
    int fc = 0;
    for (int k = o->niter - 1; k >= 0; --k) {
        if (cl) {
            int cc = 0;
            {
                ArrayList z{};
                z.add(w.lthc);
                z.add(w.lthct);
                z.add(w.lfict);
                z.add(w.lfect);
                z.add(w.lfc[cc][0]);
                z.add(w.lfc[cc][1]);
                z.add(w.ltau);
                HIPCHK(launch_zero_n(z, (long long)nca, st));
            }
            // D^T
            HIPCHK(launch_interp_adj(pf, pc, Pfc, fl->nnodes, cl->nnodes, w.lthf, w.lff[fc][0], w.lff[fc][1], w.lthc,
                                     w.lthct, w.lfc[cc][0], w.lfict, w.lfc[cc][1], w.lfect, st));
            // C^T: coarse sweeps in reverse
            const size_t cbase = 1 + (size_t)k * (Mc + nsc * Mc);
            for (int s2 = nsc - 1; s2 >= 0; --s2) {
                ArrayList z{};
                z.add(w.lfc[1 - cc][0]);
                z.add(w.lfc[1 - cc][1]);
                HIPCHK(launch_zero_n(z, (long long)nca, st));
                rc = sweep_adj_impl(cl, dt, w.tape.c + (cbase + Mc + (size_t)s2 * Mc) * nc3, w.lthc, w.lfc[cc][0],
                                    w.lfc[cc][1], w.lfc[1 - cc][0], w.lfc[1 - cc][1], w.ltau, w.tc, st);
                if (rc) return rc;
                cc = 1 - cc;
            }
            // adjoint of F at the restricted states: sweep input + saved copy
            {
                ArrayList a{};
                a.add(w.lfc[cc][0], w.lfict);
                a.add(w.lfc[cc][1], w.lfect);
                HIPCHK(launch_add_n(a, (long long)nca, st));
            }
            HIPCHK(launch_fas_tau_adj(pf, pc, PQ, Qc, fl->nnodes, cl->nnodes, dt, w.ltau, w.lff[fc][0], w.lff[fc][1],
                                      w.lfc[cc][0], w.lfc[cc][1], st));
            // B^T: restricted Theta adjoint = lthc + lthct + F^T at the restricted states
            HIPCHK(launch_add(w.lthc, w.lthct, (long long)nca, st));
            rc = tendency_adj_impl(pc, cl->p, Mc, w.tape.c + cbase * nc3, w.lfc[cc][0] + nc3, w.lfc[cc][1] + nc3,
                                   w.lthct + nc3, w.tc, st);
            if (rc) return rc;
            HIPCHK(launch_restrict_adj(pf, pc, Pcf, fl->nnodes, 1, cl->nnodes, w.lthct, w.lthf, st));
            // coarse node 0 belongs to the whole step
            {
                ArrayList a{};
                a.add(w.lthc0, w.lthct);
                a.add(w.lfic0, w.lfc[cc][0]);
                a.add(w.lfec0, w.lfc[cc][1]);
                HIPCHK(launch_add_n(a, (long long)nc3, st));
            }
        }
        // A^T: fine sweeps in reverse
        for (int s2 = nsf - 1; s2 >= 0; --s2) {
            ArrayList z{};
            z.add(w.lff[1 - fc][0]);
            z.add(w.lff[1 - fc][1]);
            HIPCHK(launch_zero_n(z, (long long)nfa, st));
            rc = sweep_adj_impl(fl, dt, w.tape.f + (1 + (size_t)(k * nsf + s2) * Mf) * nf3, w.lthf, w.lff[fc][0],
                                w.lff[fc][1], w.lff[1 - fc][0], w.lff[1 - fc][1], nullptr, w.tf, st);
            if (rc) return rc;
            fc = 1 - fc;
        }
    }
    // 3. spread^T: every fine node and its F started from Theta^n
    HIPCHK(launch_node_sum(w.lthf, lout, (long long)nf3, fl->nnodes, 0, st));
    HIPCHK(launch_node_sum(w.lff[fc][0], w.lsfi, (long long)nf3, fl->nnodes, 0, st));
    HIPCHK(launch_node_sum(w.lff[fc][1], w.lsfe, (long long)nf3, fl->nnodes, 0, st));
    rc = tendency_adj_impl(pf, fl->p, 1, w.tape.f, w.lsfi, w.lsfe, lout, w.tf, st);
    if (rc) return rc;
    if (cl) {
        rc = tendency_adj_impl(pc, cl->p, 1, w.tape.c, w.lfic0, w.lfec0, w.lthc0, w.tc, st);
        if (rc) return rc;
        Mat9x9 e0{};
        e0.a[0] = 1.0;
        HIPCHK(launch_restrict_adj(pf, pc, e0, 1, 0, 1, w.lthc0, lout, st));
    }
    return SHX_OK;
}

int sh_legendre_synthesis(const shx_plan* pl, int F, int nmax, const double* spec_ext, double* fourier,
                          shx_stream_t stream) {
    if (!pl || F < 1 || !spec_ext || !fourier || !aligned16(spec_ext) || !aligned16(fourier) ||
        (nmax != pl->N && nmax != pl->N + 1))
        return SHX_EINVAL;
    hipStream_t st = S(stream);
    HIPCHK(timed(SHX_KC_LEGENDRE_SYN, st, [&] {
        return launch_leg_syn(pl, reinterpret_cast<const double2*>(spec_ext), reinterpret_cast<double2*>(fourier), F,
                              1, nmax, st);
    }));
    return SHX_OK;
}

int sh_legendre_analysis(const shx_plan* pl, int F, int nmax, const double* fourier, double* spec_ext,
                         shx_stream_t stream) {
    if (!pl || F < 1 || !spec_ext || !fourier || !aligned16(spec_ext) || !aligned16(fourier) ||
        (nmax != pl->N && nmax != pl->N + 1))
        return SHX_EINVAL;
    hipStream_t st = S(stream);
    HIPCHK(timed(SHX_KC_LEGENDRE_AN, st, [&] {
        return launch_leg_an(pl, reinterpret_cast<const double2*>(fourier), reinterpret_cast<double2*>(spec_ext), F,
                             1, nmax, st);
    }));
    return SHX_OK;
}

size_t swe_workspace_bytes(const shx_plan* pl, int nstate) {
    if (!pl || nstate < 1) return 0;
    return tend_bytes(pl, nstate);
}

int swe_tendency(const shx_plan* pl, const swe_params* prm, int nst, const double* state, double* fi,
                 double* fe, void* ws, size_t wsb, shx_stream_t stream) {
    if (!pl || !valid_params(prm) || nst < 1 || !state || !aligned16(state) || !aligned16(fi) ||
        !aligned16(fe) || !aligned16(ws))
        return SHX_EINVAL;
    if (!alias_free(pl)) return SHX_ESHAPE;
    if (fe && (!ws || wsb < tend_bytes(pl, nst))) return SHX_EWORKSPACE;
    if (!fi && !fe) return SHX_OK;
    Carve c{static_cast<char*>(ws)};
    TendWS t = carve_tend(c, pl, nst);
    return tendency_impl(pl, *prm, nst, reinterpret_cast<const double2*>(state),
                         reinterpret_cast<double2*>(fi), reinterpret_cast<double2*>(fe), t, S(stream));
}

int imex_solve(const shx_plan* pl, const swe_params* prm, int nst, double h, const double* rhs, double* out,
               shx_stream_t stream) {
    if (!pl || !valid_params(prm) || nst < 1 || !rhs || !out || !(h >= 0.0) || !aligned16(rhs) ||
        !aligned16(out))
        return SHX_EINVAL;
    HIPCHK(launch_imex_solve(pl, *prm, h, reinterpret_cast<const double2*>(rhs), reinterpret_cast<double2*>(out),
                             nst, S(stream)));
    return SHX_OK;
}

int sdc_level_create(const shx_plan* pl, const swe_params* prm, int kind, int nnodes, sdc_level** out) {
    if (!out) return SHX_EINVAL;
    *out = nullptr;
    if (!pl || !valid_params(prm) || (kind != SDC_GAUSS_LOBATTO && kind != SDC_RADAU_RIGHT) || nnodes < 2 ||
        nnodes > 9)
        return SHX_EINVAL;
    if (kind == SDC_RADAU_RIGHT && nnodes < 3) return SHX_EINVAL;
    sdc_level* lv = new (std::nothrow) sdc_level();
    if (!lv) return SHX_EINVAL;
    lv->plan = pl;
    lv->p = *prm;
    lv->kind = kind;
    lv->nnodes = nnodes;
    if (shx_host_sdc(kind, nnodes, lv->tau, lv->Q, lv->QE, lv->QD)) {
        delete lv;
        return SHX_EINVAL;
    }
    // set-up of the allocation-free step's scratch address on the plan's device
    if (!scratch_ptr(pl->dev)) {
        delete lv;
        return SHX_EHIP;
    }
    *out = lv;
    return SHX_OK;
}

void sdc_level_destroy(sdc_level* lv) { delete lv; }

int sdc_level_matrices(const sdc_level* lv, double* tau, double* Q, double* QE, double* QD) {
    if (!lv) return SHX_EINVAL;
    const int n = lv->nnodes;
    for (int i = 0; i < n; ++i) {
        if (tau) tau[i] = lv->tau[i];
        for (int j = 0; j < n; ++j) {
            if (Q) Q[i * n + j] = lv->Q[i * n + j];
            if (QE) QE[i * n + j] = lv->QE[i * n + j];
            if (QD) QD[i * n + j] = lv->QD[i * n + j];
        }
    }
    return SHX_OK;
}

size_t sdc_sweep_workspace_bytes(const sdc_level* lv) {
    if (!lv) return 0;
    Carve c{nullptr};
    carve_sweep(c, lv);
    return c.used;
}

int sdc_sweep(const sdc_level* lv, double dt, double* th, double* fi, double* fe, const double* tau, void* ws,
              size_t wsb, shx_stream_t stream) {
    if (!lv || !th || !fi || !fe || !(dt > 0.0) || !aligned16(th) || !aligned16(fi) || !aligned16(fe) ||
        !aligned16(tau) || !aligned16(ws))
        return SHX_EINVAL;
    if (!alias_free(lv->plan)) return SHX_ESHAPE;
    if (!ws || wsb < sdc_sweep_workspace_bytes(lv)) return SHX_EWORKSPACE;
    Carve c{static_cast<char*>(ws)};
    SweepWS w = carve_sweep(c, lv);
    hipStream_t st = S(stream);
    const size_t nb = (size_t)lv->nnodes * 3 * lv->plan->nspec * sizeof(double2);
    HIPCHK(hipMemcpyAsync(w.fi_old, fi, nb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(w.fe_old, fe, nb, hipMemcpyDeviceToDevice, st));
    return sweep_impl(lv, dt, reinterpret_cast<double2*>(th), w.fi_old, w.fe_old, reinterpret_cast<double2*>(fi),
                      reinterpret_cast<double2*>(fe), reinterpret_cast<const double2*>(tau), w.t, st);
}

size_t mlsdc_workspace_bytes(const sdc_level* f, const sdc_level* c, const mlsdc_opts* o) {
    if (!f) return 0;
    Carve cv{nullptr};
    carve_step(cv, f, c, o);
    return cv.used;
}

int mlsdc_step(const sdc_level* fl, const sdc_level* cl, const mlsdc_opts* o, double dt, const double* theta_n,
               double* theta_np1, double* status, void* ws, size_t wsb, shx_stream_t stream) {
    if (!fl || !o || !theta_n || !theta_np1 || !(dt > 0.0) || o->niter < 0 || o->nsweep_fine < 1 ||
        (cl && o->nsweep_coarse < 1) || !aligned16(theta_n) || !aligned16(theta_np1) || !aligned16(ws) ||
        !aligned16(status))
        return SHX_EINVAL;
    if (cl && (cl->kind != fl->kind || cl->plan->N > fl->plan->N || cl->nnodes > fl->nnodes))
        return SHX_EINVAL;
    if (!alias_free(fl->plan) || (cl && !alias_free(cl->plan))) return SHX_ESHAPE;
    if (!ws || wsb < mlsdc_workspace_bytes(fl, cl, o)) return SHX_EWORKSPACE;
    Carve cv{static_cast<char*>(ws)};
    StepWS w = carve_step(cv, fl, cl, o);
    hipStream_t st = S(stream);
    return step_body(fl, cl, o, dt, reinterpret_cast<const double2*>(theta_n), reinterpret_cast<double2*>(theta_np1),
                     status, w, nullptr, st);
}

int mlsdc_step_noalloc(const sdc_level* fl, const sdc_level* cl, const mlsdc_opts* o, double dt,
                       const double* theta_n, double* theta_np1, double* status, shx_stream_t stream) {
    if (!fl) return SHX_EINVAL;
    const size_t need = mlsdc_workspace_bytes(fl, cl, o);
    if (need > (size_t)SHX_NOALLOC_SCRATCH_BYTES) return SHX_EWORKSPACE;
    void* ptr = scratch_ptr(fl->plan->dev);
    if (!ptr) return SHX_EHIP;
    // the same launches as mlsdc_step, on the device's scratch array
    return mlsdc_step(fl, cl, o, dt, theta_n, theta_np1, status, ptr, (size_t)SHX_NOALLOC_SCRATCH_BYTES, stream);
}

size_t mlsdc_multi_workspace_bytes(const sdc_level* const* levels, int nlevels) {
    if (!valid_levels(levels, nlevels)) return 0;
    Carve cv{nullptr};
    for (int l = 0; l < nlevels; ++l) carve_level(cv, levels[l], l == 0);
    return cv.used;
}

int mlsdc_step_multi(const sdc_level* const* levels, int nlevels, int niter, const int* nsweep, double dt,
                     const double* theta_n, double* theta_np1, void* ws, size_t wsb, shx_stream_t stream) {
    if (!valid_levels(levels, nlevels) || !nsweep || niter < 0 || !(dt > 0.0) || !theta_n || !theta_np1 ||
        !aligned16(theta_n) || !aligned16(theta_np1) || !aligned16(ws))
        return SHX_EINVAL;
    for (int l = 0; l < nlevels; ++l) {
        if (nsweep[l] < 1) return SHX_EINVAL;
        if (!alias_free(levels[l]->plan)) return SHX_ESHAPE;
    }
    if (!ws || wsb < mlsdc_multi_workspace_bytes(levels, nlevels)) return SHX_EWORKSPACE;
    Carve cv{static_cast<char*>(ws)};
    LevelWS w[SHX_MAX_LEVELS];
    for (int l = 0; l < nlevels; ++l) w[l] = carve_level(cv, levels[l], l == 0);
    return step_multi_body(levels, nlevels, niter, nsweep, dt, reinterpret_cast<const double2*>(theta_n),
                           reinterpret_cast<double2*>(theta_np1), w, S(stream));
}

}  // extern "C"
