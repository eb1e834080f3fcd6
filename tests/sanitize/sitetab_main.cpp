// Host driver for the site-local s-operator table builder (paper_1710_09621_amd/csrc/sitetab.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer.
//
// The builder is the host code with the most index arithmetic (ring neighbours, the doubling tables of the
// cyclic bidiagonal inverse).  This driver builds every table kind for every supported Ns, both chirality halves,
// a spread of masses (including m = 0 and m = 1) and weights, and checks that every entry is finite and that the
// entries past Ns stay zero; the sanitizers report any access outside the tables or undefined arithmetic.  It
// calls no HIP API.  Exit status 0 on success.
#include <cmath>
#include <cstdio>

#include "eofa_int.h"

using namespace eofa;

int main() {
    int failures = 0, built = 0;
    const int nss[] = {4, 8, 16, 32};
    const double masses[] = {0.0, 0.005, 0.1, 1.0};
    for (int Ns : nss)
        for (int w = 0; w < 2; w++) {
            double om[MAXNS];
            for (int s = 0; s < Ns; s++) {  // positive, symmetric under s -> Ns - 1 - s
                const int d = s < Ns - 1 - s ? s : Ns - 1 - s;
                om[s] = w ? 0.05 + 0.9 * d / Ns : 1.0;
            }
            for (int kind = 0; kind < SK_NKIND; kind++)
                for (double mp : masses)
                    for (double mm : masses) {
                        SiteOp op;
                        build_site_op(op, (SiteKind)kind, Ns, 1.8, om, mp, mm);
                        built++;
                        for (const ChirTab& t : op.h) {
                            const double* rows[] = {t.pre, t.mid, t.shf, t.post, t.q[0], t.q[1], t.q[2],
                                                    t.q[3], t.q[4], t.q[5]};
                            for (const double* row : rows)
                                for (int s = 0; s < MAXNS; s++) {
                                    const bool ok = s < Ns ? std::isfinite(row[s]) : row[s] == 0.0;
                                    if (!ok) {
                                        if (failures < 10)
                                            std::fprintf(stderr, "FAIL Ns=%d kind=%d mp=%g mm=%g entry %d = %g\n",
                                                         Ns, kind, mp, mm, s, row[s]);
                                        failures++;
                                    }
                                }
                        }
                    }
        }
    std::printf("site table sanitizer driver: %d tables, %d failure(s)\n", built, failures);
    return failures != 0;
}
