// Host check of the mesh look-up table (build_mesh_lut, bracket_lut in
// device_common.h) against a plain binary search over the mesh.  For every
// mesh and argument the table must give the same bracket indices and
// bitwise the same weights; a NaN argument must stay in bounds.  Exits
// non-zero on the first mismatch.  Built and run by test_mesh_lut.py.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "device_common.h"

using namespace pffrg;

namespace {

// Largest lo with w[lo] <= x, for w[0] < x < w[nf-1].
int search(const std::vector<double>& w, double x) {
    int lo = 0, hi = (int)w.size() - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (w[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

bool same(double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; }

long n_checked = 0;

bool check_mesh(const char* name, const std::vector<double>& w, std::mt19937_64& rng) {
    const int nf = (int)w.size();
    unsigned char lut[kLutMax];
    int shift = 0, kmin = 0;
    build_mesh_lut(w.data(), nf, lut, shift, kmin);
    std::vector<double> ih(nf, 0.0);
    for (int i = 0; i + 1 < nf; ++i) ih[i] = 1.0 / (w[i + 1] - w[i]);
    const MeshLut m{ih.data(), lut, shift, kmin};

    std::vector<double> xs = {0.0, 5e-324, 1e-300, w[0] * 0.5, HUGE_VAL, 1e300, w[nf - 1] * 2.0};
    for (int i = 0; i < nf; ++i) {
        xs.push_back(w[i]);
        xs.push_back(std::nextafter(w[i], 0.0));
        xs.push_back(std::nextafter(w[i], HUGE_VAL));
        if (i + 1 < nf) xs.push_back(0.5 * (w[i] + w[i + 1]));
    }
    const int nb = (int)(lut_key(w[nf - 1], shift) - lut_key(w[0], shift)) + 1;
    for (int b = 0; b <= nb; ++b) {
        const double x0 = __builtin_bit_cast(double, (unsigned long long)(kmin + b) << shift);
        xs.push_back(x0);
        xs.push_back(std::nextafter(x0, 0.0));
    }
    std::uniform_real_distribution<double> u(std::log(w[0]) - 0.1, std::log(w[nf - 1]) + 0.1);
    for (int k = 0; k < 20000; ++k) xs.push_back(std::exp(u(rng)));

    int max_steps = 0;
    for (double x : xs) {
        int i0, i1;
        double f0, f1;
        bracket_lut(w.data(), m, nf, x, i0, i1, f0, f1);
        int r0, r1;
        double g0, g1;
        if (x <= w[0]) { r0 = r1 = 0; g0 = 1.0; g1 = 0.0; }
        else if (x >= w[nf - 1]) { r0 = r1 = nf - 1; g0 = 1.0; g1 = 0.0; }
        else {
            r0 = search(w, x); r1 = r0 + 1;
            g1 = (x - w[r0]) * ih[r0];
            g0 = 1.0 - g1;
            const unsigned k = lut_key(x, shift) - (unsigned)kmin;
            if (k >= (unsigned)kLutMax) {
                std::printf("%s: x=%.17g key %u outside the table\n", name, x, k);
                return false;
            }
            if (r0 - lut[k] > max_steps) max_steps = r0 - lut[k];
        }
        if (i0 != r0 || i1 != r1 || !same(f0, g0) || !same(f1, g1)) {
            std::printf("%s: x=%.17g table (%d, %d, %.17g, %.17g) search (%d, %d, %.17g, %.17g)\n", name, x, i0,
                        i1, f0, f1, r0, r1, g0, g1);
            return false;
        }
        ++n_checked;
    }
    int i0, i1;
    double f0, f1;
    bracket_lut(w.data(), m, nf, std::nan(""), i0, i1, f0, f1);
    if (i0 < 0 || i1 < i0 || i1 >= nf) {
        std::printf("%s: NaN bracket out of bounds (%d, %d)\n", name, i0, i1);
        return false;
    }
    std::printf("%-28s nf %3d shift %d buckets %4d steps <= %d\n", name, nf, shift, nb, max_steps);
    return true;
}

std::vector<double> log_mesh(double lo, double hi, int n) {
    std::vector<double> w(n);
    for (int i = 0; i < n; ++i) w[i] = lo * std::pow(hi / lo, (double)i / (n - 1));
    return w;
}

}  // namespace

int main() {
    std::mt19937_64 rng(2109);
    bool ok = true;
    for (int n : {2, 3, 8, 24, 32, 48, 64, 128}) {
        char name[64];
        std::snprintf(name, sizeof name, "log 1e-3..100, %d", n);
        ok = ok && check_mesh(name, log_mesh(1e-3, 100.0, n), rng);
    }
    ok = ok && check_mesh("log 1e-300..1e300, 128", log_mesh(1e-300, 1e300, 128), rng);
    ok = ok && check_mesh("log 1..1.001, 128", log_mesh(1.0, 1.001, 128), rng);
    {
        std::vector<double> w(128);
        for (int i = 0; i < 128; ++i) w[i] = 0.01 + 0.1 * i;
        ok = ok && check_mesh("linear 0.01..12.7, 128", w, rng);
    }
    {
        std::vector<double> w = {1.0};
        for (int i = 1; i < 40; ++i) w.push_back(std::nextafter(w.back(), HUGE_VAL));
        ok = ok && check_mesh("adjacent doubles, 40", w, rng);
    }
    std::uniform_real_distribution<double> e(-8.0, 4.0);
    for (int t = 0; t < 20 && ok; ++t) {
        const int n = 2 + (int)(rng() % 127);
        std::vector<double> w;
        while ((int)w.size() < n) {
            const double v = std::pow(10.0, e(rng));
            bool dup = false;
            for (double q : w) dup = dup || q == v;
            if (!dup) w.push_back(v);
        }
        std::sort(w.begin(), w.end());
        ok = ok && check_mesh("random log-uniform", w, rng);
    }
    std::printf("%s: %ld arguments checked\n", ok ? "ok" : "MISMATCH", n_checked);
    return ok ? 0 : 1;
}
