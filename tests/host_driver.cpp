// CPU-only driver of libpod's host logic, built with g++ and
// -fsanitize=address,undefined by tests/test_host_sanitize.py: parameter
// validation, the POD basis (pod_compute_basis), pod_strerror, the
// neighbour-list bin geometry and the batch-assembly plan, on valid and
// invalid inputs.  Prints one line per failed check and exits non-zero on
// any failure; no HIP runtime is linked.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "pod.h"
#include "pod_plan.h"

namespace {

int failures = 0;

void check(bool ok, const char* what, int line) {
    if (!ok) {
        std::printf("FAIL line %d: %s\n", line, what);
        ++failures;
    }
}
#define CHECK(x) check((x), #x, __LINE__)

struct Family {
    std::vector<double> alpha, beta, gamma, kappa;
    pod_params p{};
};

// Standard family: nb Bessel snapshots (alpha = 1..nb, one beta) then ni
// inverse powers (gamma = 1..ni).
Family standard(int nb, int ni, int K, int P) {
    Family f;
    for (int l = 0; l < nb; ++l) {
        f.alpha.push_back(l + 1.0); f.beta.push_back(3.0); f.gamma.push_back(0.0); f.kappa.push_back(1.0);
    }
    for (int l = 0; l < ni; ++l) {
        f.alpha.push_back(0.0); f.beta.push_back(0.0); f.gamma.push_back(l + 1.0); f.kappa.push_back(0.0);
    }
    f.p.rin = 0.5; f.p.rcut = 5.0; f.p.L = nb + ni;
    f.p.alpha = f.alpha.data(); f.p.beta = f.beta.data(); f.p.gamma = f.gamma.data(); f.p.kappa = f.kappa.data();
    f.p.K2 = K; f.p.K3 = K; f.p.K4 = K; f.p.P3 = P; f.p.P4 = P;
    f.p.Q = nullptr; f.p.n_quad = 0; f.p.dtype = POD_F64;
    return f;
}

void test_strerror() {
    const int codes[] = {POD_OK, POD_EINVAL, POD_ERANGE, POD_ENONFINITE, POD_ENOMEM, POD_EHIP,
                         POD_ENOTSUP, POD_ENEIGH, POD_ESINGULAR, POD_ETOOBIG, 12345, -12345};
    for (int c : codes) {
        const char* s = pod_strerror(c);
        CHECK(s != nullptr && std::strlen(s) > 0);
    }
    CHECK(std::strcmp(pod_strerror(12345), "unknown error") == 0);
}

void test_basis() {
    for (int L : {1, 2, 8, POD_MAX_L}) {
        Family f = standard((L + 1) / 2, L / 2, 1, 0);
        f.p.n_quad = L == 8 ? 0 : 4 * L + 3;
        std::vector<double> Q(static_cast<size_t>(L) * L, -1.0), e(L, -1.0);
        CHECK(pod_compute_basis(&f.p, Q.data(), e.data()) == POD_OK);
        for (int k = 0; k + 1 < L; ++k) CHECK(e[k] >= e[k + 1]);
        for (int k = 0; k < L; ++k) CHECK(e[k] >= -1e-12 * std::fabs(e[0]));
        for (int a = 0; a < L; ++a)
            for (int b = 0; b < L; ++b) {
                double d = 0.0;
                for (int l = 0; l < L; ++l) d += Q[l * L + a] * Q[l * L + b];
                CHECK(std::fabs(d - (a == b ? 1.0 : 0.0)) < 1e-10);
            }
    }
    // null outputs are allowed
    Family f = standard(4, 4, 4, 4);
    CHECK(pod_compute_basis(&f.p, nullptr, nullptr) == POD_OK);
}

void test_validation() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    CHECK(pod::validate_params(nullptr) == POD_EINVAL);
    CHECK(pod_compute_basis(nullptr, nullptr, nullptr) == POD_EINVAL);
    {
        Family f = standard(4, 4, 6, 4);
        CHECK(pod::validate_params(&f.p) == POD_OK);
    }
    struct Case {
        const char* what;
        int expect;
        void (*edit)(Family&);
    };
    const Case cases[] = {
        {"rin >= rcut", POD_EINVAL, [](Family& f) { f.p.rin = 5.0; }},
        {"rin < 0", POD_EINVAL, [](Family& f) { f.p.rin = -0.1; }},
        {"rcut inf", POD_EINVAL, [](Family& f) { f.p.rcut = std::numeric_limits<double>::infinity(); }},
        {"L = 0", POD_EINVAL, [](Family& f) { f.p.L = 0; }},
        {"L > max", POD_ENOTSUP, [](Family& f) { f.p.L = POD_MAX_L + 1; }},
        {"alpha null", POD_EINVAL, [](Family& f) { f.p.alpha = nullptr; }},
        {"alpha nan", POD_EINVAL, [](Family& f) { f.alpha[2] = std::numeric_limits<double>::quiet_NaN(); }},
        {"kappa > 1", POD_EINVAL, [](Family& f) { f.kappa[0] = 1.5; }},
        {"beta < 0", POD_EINVAL, [](Family& f) { f.beta[1] = -1.0; }},
        {"K2 < 0", POD_EINVAL, [](Family& f) { f.p.K2 = -1; }},
        {"all K zero", POD_EINVAL, [](Family& f) { f.p.K2 = f.p.K3 = f.p.K4 = 0; }},
        {"K > L", POD_EINVAL, [](Family& f) { f.p.K3 = f.p.L + 1; }},
        {"P3 > max", POD_ENOTSUP, [](Family& f) { f.p.P3 = POD_MAX_P + 1; }},
        {"P4 > max", POD_ENOTSUP, [](Family& f) { f.p.P4 = POD_MAX_P4 + 1; }},
        {"K > max", POD_ENOTSUP, [](Family& f) {
             f.p.L = POD_MAX_L;
             f.alpha.resize(POD_MAX_L, 1.0); f.beta.resize(POD_MAX_L, 0.0);
             f.gamma.resize(POD_MAX_L, 1.0); f.kappa.resize(POD_MAX_L, 0.0);
             f.p.alpha = f.alpha.data(); f.p.beta = f.beta.data(); f.p.gamma = f.gamma.data();
             f.p.kappa = f.kappa.data();
             f.p.K4 = POD_MAX_K + 1; }},
        {"P4 < 0", POD_EINVAL, [](Family& f) { f.p.P4 = -2; }},
        {"dtype", POD_EINVAL, [](Family& f) { f.p.dtype = 7; }},
        {"n_quad < 2L", POD_EINVAL, [](Family& f) { f.p.n_quad = 3; }},
    };
    for (const Case& c : cases) {
        Family f = standard(4, 4, 6, 4);
        f.p.alpha = f.alpha.data(); f.p.beta = f.beta.data(); f.p.gamma = f.gamma.data(); f.p.kappa = f.kappa.data();
        c.edit(f);
        const int rc = pod::validate_params(&f.p);
        if (rc != c.expect) std::printf("  case %s: got %d, expected %d\n", c.what, rc, c.expect);
        CHECK(rc == c.expect);
        CHECK(pod_compute_basis(&f.p, nullptr, nullptr) == c.expect);
    }
    {
        Family f = standard(4, 4, 6, 4);
        std::vector<double> Q(8 * 6, 0.1);
        Q[17] = nan;
        f.p.Q = Q.data();
        CHECK(pod::validate_params(&f.p) == POD_EINVAL);
        Q[17] = inf;
        CHECK(pod::validate_params(&f.p) == POD_EINVAL);
        Q[17] = 0.0;
        CHECK(pod::validate_params(&f.p) == POD_OK);
    }
}

void test_periodic_geometry() {
    pod::NbGeom g{};
    const double cube[9] = {10, 0, 0, 0, 10, 0, 0, 0, 10};
    CHECK(pod::periodic_geometry(cube, 4.9, &g) == POD_OK);
    for (int d = 0; d < 3; ++d) {
        CHECK(g.nb[d] == 2 && g.ns[d] == 1);
        CHECK(10.0 / g.nb[d] >= 4.9);                 // bins at least r_list wide
    }
    // r_list exactly half the cell: the search widens by one bin rather than
    // trusting the rounding of 10 / 2 == 5
    CHECK(pod::periodic_geometry(cube, 5.0, &g) == POD_OK);
    for (int d = 0; d < 3; ++d) CHECK(g.nb[d] == 2 && g.ns[d] == 2);
    // inverse: a inv = I
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += g.a[3 * i + k] * g.inv[3 * k + j];
            CHECK(std::fabs(s - (i == j ? 1.0 : 0.0)) < 1e-14);
        }
    // triclinic cell thinner than r_list in one direction: one bin there,
    // searched over enough bins to cover r_list
    const double tri[9] = {3.4, 0, 0, 0.9, 3.2, 0, 0.4, 0.6, 3.6};
    CHECK(pod::periodic_geometry(tri, 4.5, &g) == POD_OK);
    for (int d = 0; d < 3; ++d) CHECK(g.nb[d] >= 1 && g.ns[d] >= 2);
    // large cell: bins capped at NB_MAX_BINS per direction
    const double big[9] = {1e4, 0, 0, 0, 1e4, 0, 0, 0, 1e4};
    CHECK(pod::periodic_geometry(big, 5.0, &g) == POD_OK);
    for (int d = 0; d < 3; ++d) CHECK(g.nb[d] == pod::NB_MAX_BINS && g.ns[d] * 1e4 / g.nb[d] >= 5.0);
    // a cell so thin that the search would span too many bins
    const double thin[9] = {10, 0, 0, 0, 10, 0, 0, 0, 0.05};
    CHECK(pod::periodic_geometry(thin, 5.0, &g) == POD_ENOTSUP);
    const double sing[9] = {1, 0, 0, 2, 0, 0, 0, 0, 1};
    CHECK(pod::periodic_geometry(sing, 5.0, &g) == POD_EINVAL);
    double bad[9] = {10, 0, 0, 0, 10, 0, 0, 0, 10};
    bad[4] = std::numeric_limits<double>::quiet_NaN();
    CHECK(pod::periodic_geometry(bad, 5.0, &g) == POD_EINVAL);
    CHECK(pod::periodic_geometry(cube, 0.0, &g) == POD_EINVAL);
    CHECK(pod::periodic_geometry(cube, -1.0, &g) == POD_EINVAL);
    CHECK(pod::periodic_geometry(nullptr, 5.0, &g) == POD_EINVAL);
}

void test_open_geometry() {
    pod::NbGeom g{};
    CHECK(pod::open_geometry(nullptr, 0, 5.0, &g) == POD_OK);
    for (int d = 0; d < 3; ++d) CHECK(g.nb[d] == 1);
    std::vector<double> pos = {0, 0, 0, 12, 1, 2, 3, 4, 20};
    CHECK(pod::open_geometry(pos.data(), 3, 5.0, &g) == POD_OK);
    CHECK(g.nb[0] == 3 && g.nb[1] == 1 && g.nb[2] == 5);
    for (int d = 0; d < 3; ++d) CHECK(g.bw[d] >= 5.0 && g.bw[d] * g.nb[d] >= (d == 0 ? 12.0 : d == 1 ? 4.0 : 20.0));
    // non-finite coordinates are skipped here (the bin kernel latches them)
    pos[4] = std::numeric_limits<double>::quiet_NaN();
    pos[0] = std::numeric_limits<double>::infinity();
    CHECK(pod::open_geometry(pos.data(), 3, 5.0, &g) == POD_OK);
    // extent so large that ext / r_list overflows the bin count: capped
    std::vector<double> far = {-1e300, 0, 0, 1e300, 0, 0};
    CHECK(pod::open_geometry(far.data(), 2, 1e-300, &g) == POD_OK);
    CHECK(g.nb[0] == pod::NB_MAX_BINS);
    CHECK(pod::open_geometry(pos.data(), -1, 5.0, &g) == POD_EINVAL);
    CHECK(pod::open_geometry(pos.data(), 3, std::numeric_limits<double>::quiet_NaN(), &g) == POD_EINVAL);
}

void test_batch_plan() {
    // 4 cells of 2, 3, 1, 2 atoms; pair counts 3, 9, 0, 3
    const std::vector<int> coff = {0, 2, 5, 6, 8};
    const std::vector<int> off = {0, 1, 3, 6, 9, 12, 12, 14, 15};
    pod::BatchPlan plan;
    CHECK(pod::plan_batch(4, 8, 15, coff.data(), off.data(), 37, 64 * 1024, nullptr, &plan) == POD_OK);
    CHECK(plan.max_nc == 3 && plan.max_pc == 9 && plan.nc_max == 16);
    CHECK(plan.cw == 17 && plan.nth == 512 && plan.nblk == 4);
    CHECK(plan.lds == pod::batch_lds(37, 17, 16).total);
    CHECK((plan.order == std::vector<int>{1, 0, 3, 2}));   // decreasing pairs, ties keep order
    // tuning: chunk width reduced until the LDS layout fits
    pod_tune t{};
    t.cw = 64; t.nblocks = 2; t.threads = 256;
    const size_t cap = pod::batch_lds(37, 9, 16).total;
    CHECK(pod::plan_batch(4, 8, 15, coff.data(), off.data(), 37, cap, &t, &plan) == POD_OK);
    CHECK(plan.cw == 9 && plan.nblk == 2 && plan.nth == 256 && plan.lds <= cap);
    CHECK(pod::plan_batch(4, 8, 15, coff.data(), off.data(), 37, 64, &t, &plan) == POD_ENOTSUP);
    t.threads = 100;
    CHECK(pod::plan_batch(4, 8, 15, coff.data(), off.data(), 37, 64 * 1024, &t, &plan) == POD_EINVAL);
    t.threads = 1024;
    CHECK(pod::plan_batch(4, 8, 15, coff.data(), off.data(), 37, 64 * 1024, &t, &plan) == POD_EINVAL);
    // malformed offsets
    std::vector<int> c2 = coff;
    c2[2] = 1;                                   // cells overlap
    CHECK(pod::plan_batch(4, 8, 15, c2.data(), off.data(), 37, 64 * 1024, nullptr, &plan) == POD_EINVAL);
    c2 = coff;
    c2[1] = 100;                                 // beyond N: refused before any read past off[N]
    CHECK(pod::plan_batch(4, 8, 15, c2.data(), off.data(), 37, 64 * 1024, nullptr, &plan) == POD_EINVAL);
    c2 = coff;
    c2[4] = 7;                                   // does not end at N
    CHECK(pod::plan_batch(4, 8, 15, c2.data(), off.data(), 37, 64 * 1024, nullptr, &plan) == POD_EINVAL);
    std::vector<int> o2 = off;
    o2[3] = 2;                                   // pair offsets decrease
    CHECK(pod::plan_batch(4, 8, 15, coff.data(), o2.data(), 37, 64 * 1024, nullptr, &plan) == POD_ENEIGH);
    CHECK(pod::plan_batch(4, 8, 14, coff.data(), off.data(), 37, 64 * 1024, nullptr, &plan) == POD_EINVAL);
    CHECK(pod::plan_batch(0, 8, 15, coff.data(), off.data(), 37, 64 * 1024, nullptr, &plan) == POD_EINVAL);
    CHECK(pod::plan_batch(4, 8, 15, nullptr, off.data(), 37, 64 * 1024, nullptr, &plan) == POD_EINVAL);
}

}  // namespace

int main() {
    test_strerror();
    test_basis();
    test_validation();
    test_periodic_geometry();
    test_open_geometry();
    test_batch_plan();
    if (failures == 0) std::printf("host driver: all checks passed\n");
    return failures == 0 ? 0 : 1;
}
