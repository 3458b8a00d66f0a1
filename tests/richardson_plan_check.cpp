// Host-only check of the Chebyshev-Richardson plan (no GPU) against its
// closed form.  For each interval [lo, hi] and tolerance given on the command
// line as lo,hi,tol triples:
//   - the plan's step roots theta (1/g0 and 1/tau_k) are the d roots of T_d
//     mapped onto [lo, hi], each once;
//   - the first root is the one of largest magnitude and every later one
//     maximises the product of its distances to the roots before it (Leja);
//   - the plan reports 1/T_d(c/h), and (for d <= 100) the residual polynomial
//     prod_k (1 - lambda/theta_k) of the iteration, evaluated on a fine grid of
//     [lo, hi] with its ends, stays within that factor and reaches it;
//   - d is the smallest degree (>= 3) whose 1/T_d(c/h) meets tol; a plan
//     capped at kRichMaxDegree reports the factor it reaches (above tol).
// Prints "ok d reached maxres" per case and exits 0, or names the first failure.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.h"

int main(int argc, char** argv) {
    for (int a = 1; a < argc; ++a) {
        double lo = 0, hi = 0, tol = 0;
        if (sscanf(argv[a], "%lf,%lf,%lf", &lo, &hi, &tol) != 3) return 2;
        const elses::Rich r = elses::richardson_plan(lo, hi, tol);
        const int d = r.d;
        if ((int)r.tau.size() != d - 1) {
            printf("FAIL %s: %zu inverse roots for degree %d\n", argv[a], r.tau.size(), d);
            return 1;
        }
        std::vector<double> th(d);
        th[0] = 1.0 / r.g0;
        for (int k = 1; k < d; ++k) th[k] = 1.0 / r.tau[k - 1];
        // the roots of T_d on [lo, hi]
        const double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo);
        std::vector<double> want(d), got(th);
        for (int i = 0; i < d; ++i) want[i] = c + h * std::cos(M_PI * (2.0 * i + 1.0) / (2.0 * d));
        std::sort(want.begin(), want.end());
        std::sort(got.begin(), got.end());
        for (int i = 0; i < d; ++i)
            if (std::fabs(want[i] - got[i]) > 1e-12 * hi) {
                printf("FAIL %s: root %d is %.17g, not %.17g\n", argv[a], i, got[i], want[i]);
                return 1;
            }
        // Leja order
        for (int i = 1; i < d; ++i)
            if (std::fabs(th[i]) > std::fabs(th[0])) {
                printf("FAIL %s: first root is not the largest\n", argv[a]);
                return 1;
            }
        for (int k = 1; k < d; ++k) {
            auto score = [&](double x) {
                double p = 0.0;
                for (int j = 0; j < k; ++j) p += std::log(std::fabs(x - th[j]));
                return p;
            };
            const double mine = score(th[k]);
            for (int i = k + 1; i < d; ++i)
                if (score(th[i]) > mine + 1e-9) {
                    printf("FAIL %s: step %d is not the Leja choice\n", argv[a], k);
                    return 1;
                }
        }
        // residual polynomial on [lo, hi] against 1/T_d(c/h)
        const double sigma = c / h;
        const double bound = 1.0 / std::cosh(d * std::acosh(sigma));
        if (std::fabs(r.reached - bound) > 1e-9 * bound) {
            printf("FAIL %s: reported factor %.6g, closed form %.6g\n", argv[a], r.reached, bound);
            return 1;
        }
        double maxres = bound;
        const int n = d <= 100 ? 40001 : 0;  // (a long product's rounding outgrows tiny factors)
        if (n) maxres = 0.0;
        for (int i = 0; i < n; ++i) {
            const double lam = lo + (hi - lo) * i / (n - 1);
            double p = 1.0;
            for (int k = 0; k < d; ++k) p *= 1.0 - lam / th[k];
            maxres = std::max(maxres, std::fabs(p));
        }
        if (maxres > bound * (1.0 + 1e-6) || maxres < bound * (1.0 - 1e-3)) {
            printf("FAIL %s: max residual factor %.6g on the interval, bound %.6g\n", argv[a], maxres, bound);
            return 1;
        }
        // minimal degree, or the cap
        if (d == elses::kRichMaxDegree && !(bound > tol)) {
            printf("FAIL %s: capped although degree %d reaches tol\n", argv[a], d);
            return 1;
        }
        if (d < elses::kRichMaxDegree) {
            if (bound > tol * (1.0 + 1e-12)) {
                printf("FAIL %s: degree %d reaches %.3g > tol\n", argv[a], d, bound);
                return 1;
            }
            if (d > 3 && 1.0 / std::cosh((d - 1) * std::acosh(sigma)) <= tol) {
                printf("FAIL %s: degree %d is not the smallest\n", argv[a], d);
                return 1;
            }
        }
        printf("ok %d %.6g %.6g\n", d, r.reached, maxres);
    }
    return 0;
}
