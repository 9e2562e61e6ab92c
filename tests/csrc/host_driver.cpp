// Host-only driver of the library's C ABI for the sanitizer test: every call
// here runs on the CPU (validation, step sizes, workspace sizes, the static
// entry point's refusal), so it runs without a GPU.  Exit status 0 when every
// call returned what it should.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "omt.h"
#include "omt_matrix.h"

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, omt_last_error());
        ++failures;
    }
}

int main()
{
    const int32_t tri[6] = {0, 1, 0, 2, 1, 2};
    const int32_t path8[14] = {0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6, 6, 7};
    const double costs[3] = {1.0, 2.0, 0.5};
    double h, mu, nu, lam;
    size_t bytes = 0;

    // valid problems of every compiled kind, 2-D and 3-D, both dtypes
    for (int dt = 0; dt < 2; ++dt)
        for (int k = 1; k <= 8; ++k) {
            omt_params p;
            omt_params_init(&p);
            p.m = 37 + k;
            p.n = 129 - k;
            p.k = k;
            p.dtype = dt;
            p.n_edges = k >= 2 ? (k == 3 ? 3 : k - 1) : 0;
            p.edges = k == 3 ? tri : path8;
            p.edge_cost = k == 3 ? costs : nullptr;
            p.unorm = k % 3;
            p.wnorm = k % 2;
            p.reg_eps = k == 4 ? 0.01 : 0.0;
            expect(omt_resolve_params(&p, &h, &mu, &nu, &lam) == OMT_OK, "resolve 2-D");
            expect(std::fabs(h - 1.0 / (p.m - 1 > p.n - 1 ? p.m - 1 : p.n - 1)) < 1e-15, "h rule");
            expect(omt_workspace_bytes(&p, &bytes) == OMT_OK && bytes > 0, "workspace 2-D");
            if (k <= 3) {
                p.p = 5 + k;
                const omt_status s = omt_resolve_params(&p, &h, &mu, &nu, &lam);
                expect(s == OMT_OK || s == OMT_EUNSUPPORTED, "resolve 3-D");
                if (s == OMT_OK) expect(omt_workspace_bytes(&p, &bytes) == OMT_OK && bytes > 0, "workspace 3-D");
            }
        }

    // invalid requests are refused with the documented status
    {
        omt_params p;
        omt_params_init(&p);
        p.m = 1;
        p.n = 10;
        p.k = 1;
        expect(omt_resolve_params(&p, &h, &mu, &nu, &lam) == OMT_EINVAL, "m < 2");
        p.m = 10;
        p.k = 3;
        const int32_t bad[2] = {1, 1};
        p.n_edges = 1;
        p.edges = bad;
        expect(omt_resolve_params(&p, &h, &mu, &nu, &lam) == OMT_EGRAPH, "self loop");
        p.edges = tri;
        p.n_edges = 3;
        p.mu = 1.0;
        p.nu = 1.0;
        expect(omt_resolve_params(&p, &h, &mu, &nu, &lam) == OMT_ESTEP, "steps too large");
        p.mu = p.nu = 0.0;
        p.k = 9;
        const omt_status s9 = omt_resolve_params(&p, &h, &mu, &nu, &lam);
        expect(s9 == OMT_EINVAL || s9 == OMT_EUNSUPPORTED, "k = 9");
        p.k = 3;
        p.tau = -1.0;
        expect(omt_resolve_params(&p, &h, &mu, &nu, &lam) == OMT_EINVAL, "tau < 0");
    }

    // batch sizes, and the static entry point refusing an oversize problem
    {
        omt_params ps[3];
        for (int q = 0; q < 3; ++q) {
            omt_params_init(&ps[q]);
            ps[q].m = 64 + 17 * q;
            ps[q].n = 90 - 11 * q;
            ps[q].k = q == 2 ? 3 : 1;
            ps[q].n_edges = q == 2 ? 3 : 0;
            ps[q].edges = tri;
        }
        expect(omt_batch_workspace_bytes(3, ps, &bytes) == OMT_OK && bytes > 0, "batch workspace");
        expect(omt_batch_workspace_bytes(0, ps, &bytes) == OMT_EINVAL, "empty batch");
        omt_params big;
        omt_params_init(&big);
        big.m = big.n = 1024;
        big.k = 3;
        big.n_edges = 3;
        big.edges = tri;
        expect(omt_solve_static(&big, nullptr, nullptr, 10, 0.0, 64, nullptr, nullptr, nullptr, nullptr, nullptr) ==
                   OMT_ENOMEM,
               "static oversize");
    }

    // matrix problems: real 3 x 3 with two L, complex 2 x 2, and a bad L
    {
        omt_matrix_params p;
        omt_matrix_params_init(&p);
        double L[2 * 9 * 2];
        std::memset(L, 0, sizeof(L));
        // L1 = diag(1, 0, -1); L2 = symmetric with ones off the diagonal
        L[(0 * 3 + 0) * 2] = 1.0;
        L[(2 * 3 + 2) * 2] = -1.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (a != b) L[(9 + a * 3 + b) * 2] = 1.0;
        p.m = 40;
        p.n = 70;
        p.k = 3;
        p.n_L = 2;
        p.L = L;
        p.real = 1;
        int32_t nc = 0, nw = 0;
        expect(omt_matrix_resolve(&p, &h, &mu, &nu, &lam, &nc, &nw) == OMT_OK && nc == 6, "matrix real 3x3");
        expect(omt_matrix_workspace_bytes(&p, &bytes) == OMT_OK && bytes > 0, "matrix workspace");
        L[(0 * 3 + 1) * 2] = 5.0;  // L1 no longer symmetric
        expect(omt_matrix_resolve(&p, &h, &mu, &nu, &lam, &nc, &nw) == OMT_EINVAL, "non-Hermitian L");
    }

    for (int s = 0; s <= 9; ++s) expect(omt_strerror(static_cast<omt_status>(s))[0] != 0, "strerror");
    std::printf("host driver: %d failure(s)\n", failures);
    return failures == 0 ? 0 : 1;
}
