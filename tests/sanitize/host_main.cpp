// Exercises the library's host runtime under AddressSanitizer and
// UndefinedBehaviorSanitizer, with no GPU: the Revolve schedule (both split rules), its
// step counts, the profile planner, the run-time model and the strategy choice (which
// replay the executor's bookkeeping host-side), and the set-up of solo and batched
// calls (validation, source and receiver tables, workspace layout).  Any sanitizer
// report aborts with a non-zero status; the run prints OK at the end.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/wv.h"

static void fail(const char *what)
{
    std::fprintf(stderr, "FAILED: %s\n", what);
    std::exit(1);
}

int main()
{
    // schedules
    for (int nt : {1, 2, 3, 7, 50, 333, 1000}) {
        for (int M : {1, 2, 3, 5, 17, 64, 1000}) {
            for (int wm = 0; wm < 2; ++wm) {
                size_t n = 0;
                wv_schedule(nt, M, wm, nullptr, 0, &n);
                std::vector<int32_t> a(3 * (n + 1));
                if (wv_schedule(nt, M, wm, a.data(), n, &n) != WV_OK) fail("wv_schedule");
                long adv = 0, rev = 0;
                for (size_t i = 0; i < n; ++i) {
                    if (a[3 * i] == 1) adv += a[3 * i + 2] - a[3 * i + 1];
                    if (a[3 * i] == 5) ++rev;
                }
                if (adv != wv_schedule_forward_steps(nt, M) || rev != nt) fail("schedule counts");
            }
        }
    }
    // planner, model and choice on a synthetic growing profile
    double prof[WV_PROFILE];
    for (int j = 0; j < WV_PROFILE; ++j) prof[j] = 1e5 + 4e6 * j;
    wv_costs cp{0.2, 0.45, 0.09, 0.0, 0.0, 1.0, 0.0}, cc{0.2, 0.45, 0.0, 0.13, 0.07, 20.0, 0.0};
    for (size_t budget : {size_t(0), size_t(1) << 20, size_t(2e9), size_t(16e9), size_t(1e12)}) {
        int M = 0;
        double hint = 0.0;
        if (wv_plan(3000, 64000000LL, budget, prof, WV_PROFILE, &M, &hint) != WV_OK || M < 1) fail("wv_plan");
        wv_prediction p{};
        if (wv_predict(3000, 64000000LL, budget, 0, &cp, &p) != WV_OK) fail("wv_predict plain");
        if (wv_predict(3000, 64000000LL, budget, 1, &cc, &p) != WV_OK) fail("wv_predict compressed");
        wv_choice ch{};
        if (wv_choose(3000, 64000000LL, budget, &cp, &cc, prof, WV_PROFILE, &ch) != WV_OK) fail("wv_choose");
    }
    // set-up of solo and batched calls (no device work: queries only)
    const float *fake = reinterpret_cast<const float *>(0x1000);
    for (int nd = 2; nd <= 3; ++nd) {
        for (int order : {2, 8, 16}) {
            wv_model m{};
            m.ndim = nd;
            m.n[0] = 37; m.n[1] = nd == 3 ? 29 : 41; m.n[2] = nd == 3 ? 23 : 1;
            m.h[0] = m.h[1] = m.h[2] = 10.0;
            m.nbl = 7; m.space_order = order; m.nt = 120; m.vmax = 3000.0; m.vel = fake; m.time_order = 2;
            m.dt = 0.4 * wv_cfl_dt(nd, m.h, order, m.vmax);
            std::vector<double> src = {180.0, 100.0, 20.0}, rec;
            for (int r = 0; r < 37; ++r) {
                rec.push_back(10.0 * r);
                rec.push_back(nd == 3 ? 50.0 : 20.0);
                if (nd == 3) rec.push_back(20.0);
            }
            wv_geom g{1, src.data(), fake, 37, rec.data()};
            if (wv_field_elements(&m) <= 0) fail("wv_field_elements");
            for (int op = 0; op < 3; ++op)
                if (wv_workspace_bytes(&m, &g, op, size_t(1) << 24) == 0) fail("wv_workspace_bytes");
            if (nd == 2) {
                std::vector<wv_model> ms(5, m);
                std::vector<wv_geom> gs(5, g);
                if (wv_batch_workspace_bytes(5, ms.data(), gs.data(), size_t(1) << 24) == 0) fail("batch workspace");
                ms[3].nt = 121;   // not batchable with the others
                if (wv_batch_workspace_bytes(5, ms.data(), gs.data(), size_t(1) << 24) != 0) fail("batch check");
            }
        }
    }
    std::printf("OK\n");
    return 0;
}
