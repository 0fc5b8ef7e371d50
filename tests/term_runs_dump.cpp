// Splits pair term lists into runs with term_runs (csrc/kernels_flow.h),
// host build, for tests/test_term_runs.py.  Reads cases from stdin, one per
// line: ns off[0] .. off[ns]; prints per case
//   N nrun
//   R r x y        for every r < 64
//   O p run_off    for every p <= ns
#include <cstdio>
#include <vector>

#include "kernels_flow.h"

int main() {
    int ns;
    while (std::scanf("%d", &ns) == 1) {
        std::vector<int> off(ns + 1), run(2 * pffrg::kWave), run_off(ns + 1);
        for (int p = 0; p <= ns; ++p)
            if (std::scanf("%d", &off[p]) != 1) return 1;
        const int n = pffrg::term_runs(ns, off.data(), run.data(), run_off.data());
        std::printf("N %d\n", n);
        for (int r = 0; r < pffrg::kWave; ++r) std::printf("R %d %d %d\n", r, run[2 * r], run[2 * r + 1]);
        for (int p = 0; p <= ns; ++p) std::printf("O %d %d\n", p, run_off[p]);
    }
    return 0;
}
