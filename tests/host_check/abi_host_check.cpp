// Host-side checks of the library built with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code: the quad-precision set-up
// routines (Gaussian latitudes, SDC matrices, transfer matrices, twiddles,
// working-precision values) and the synchronous argument validation of the C
// ABI, none of which touches a GPU.  Exits 0 when every check holds (a
// sanitizer report aborts the run).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/mlsdc_sh.h"
#include "../../paper_1805_07923_amd/csrc/setup_host.h"

static int g_fail = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

int main() {
    // Gaussian latitudes: weights sum to 2, nodes antisymmetric, 1 - mu^2 = sin^2
    for (int J : {2, 3, 48, 96, 384, 1536}) {
        std::vector<double> mu(J), st(J), c2(J), w(J);
        CHECK(shx_host_gauss(J, mu.data(), st.data(), c2.data(), w.data()) == 0);
        double sw = 0.0;
        for (int j = 0; j < J; ++j) {
            sw += w[j];
            CHECK(std::fabs(mu[j] + mu[J - 1 - j]) <= 1e-15);
            CHECK(std::fabs(c2[j] - st[j] * st[j]) <= 1e-15);
            if (j > 0) CHECK(mu[j] < mu[j - 1]);
        }
        CHECK(std::fabs(sw - 2.0) <= 1e-13);
    }
    // SDC matrices: row m of Q integrates 1 to tau_m; Q_E, Q_Delta lower triangular
    for (int kind : {0, 1})
        for (int n = (kind ? 3 : 2); n <= 9; ++n) {
            double tau[9], Q[81], QE[81], QD[81];
            CHECK(shx_host_sdc(kind, n, tau, Q, QE, QD) == 0);
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) {
                    s += Q[i * n + j];
                    if (j > i) CHECK(QE[i * n + j] == 0.0 && QD[i * n + j] == 0.0);
                }
                CHECK(std::fabs(s - tau[i]) <= 1e-14);
            }
            // transfer matrices between node sets: rows sum to 1 (constants are interpolated exactly)
            for (int nc = (kind ? 3 : 2); nc <= n; ++nc) {
                double P[81];
                CHECK(shx_host_transfer(kind, n, nc, P) == 0);
                for (int i = 0; i < nc; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < n; ++j) s += P[i * n + j];
                    CHECK(std::fabs(s - 1.0) <= 1e-13);
                }
            }
        }
    // twiddles on the unit circle
    for (int L : {16, 48, 768, 3072}) {
        std::vector<double> re(L), im(L);
        shx_host_twiddles(L, re.data(), im.data());
        for (int t = 0; t < L; ++t) CHECK(std::fabs(re[t] * re[t] + im[t] * im[t] - 1.0) <= 4e-16);
    }
    // working-precision values
    CHECK(shx_host_working_value(0, 0.1) == 0.1);
    CHECK(shx_host_working_value(1, 0.1) == (double)(float)0.1);
    CHECK(std::fabs(shx_host_working_value(2, 0.1) - 0.1) <= 1e-5);
    CHECK(std::fabs(shx_host_working_value(3, 0.1) - 0.1) <= 1e-7);
    // argument validation of the ABI (returns before any device work)
    shx_plan* h = nullptr;
    CHECK(shx_plan_create(31, 48, 96, 0, 0, nullptr) == SHX_EINVAL);
    CHECK(shx_plan_create(0, 48, 96, 0, 0, &h) == SHX_EINVAL);
    CHECK(shx_plan_create(31, 48, 96, 0, 7, &h) == SHX_EINVAL);
    CHECK(shx_plan_create(31, 47, 96, 0, 0, &h) == SHX_ESHAPE);
    CHECK(shx_plan_create(31, 48, 62, 0, 0, &h) == SHX_ESHAPE);
    CHECK(shx_plan_create(31, 48, 100, 0, 0, &h) == SHX_EUNSUPPORTED);
    CHECK(shx_plan_create(31, 48, 96, 9, 0, &h) == SHX_EUNSUPPORTED);
    CHECK(h == nullptr);
    CHECK(shx_nspec(31) == 32 * 33 / 2);
    CHECK(shx_nspec(-1) == 0);
    swe_params par{6.37122e6, 7.292e-5, 9.80616, 2.94e4, 1e5};
    sdc_level* lv = nullptr;
    CHECK(sdc_level_create(nullptr, &par, 0, 3, &lv) == SHX_EINVAL);
    CHECK(sh_inverse(nullptr, 1, nullptr, nullptr, nullptr, 0, nullptr) == SHX_EINVAL);
    CHECK(sh_forward(nullptr, 1, nullptr, nullptr, nullptr, 0, nullptr) == SHX_EINVAL);
    long long terms = 0;
    CHECK(shx_plan_analysis_terms(nullptr, 31, &terms, nullptr) == SHX_EINVAL);
    CHECK(swe_tendency(nullptr, &par, 1, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == SHX_EINVAL);
    CHECK(mlsdc_step(nullptr, nullptr, nullptr, 1.0, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == SHX_EINVAL);
    CHECK(mlsdc_step_noalloc(nullptr, nullptr, nullptr, 1.0, nullptr, nullptr, nullptr, nullptr) == SHX_EINVAL);
    CHECK(mlsdc_step_adj(nullptr, nullptr, nullptr, 1.0, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
          SHX_EINVAL);
    CHECK(mlsdc_workspace_bytes(nullptr, nullptr, nullptr) == 0);
    for (int c = 0; c >= -6; --c) CHECK(shx_strerror(c) != nullptr && std::strlen(shx_strerror(c)) > 0);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
