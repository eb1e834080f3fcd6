/*
 * Host driver for the FP64 oracle (oracle/oracle.c) under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Test infrastructure only: it calls every exported oracle function on small lattices (with a dimension of 2,
 * odd and even Ns, both chiralities, both directions) so that an out-of-bounds access, a use after free, a leak
 * or undefined arithmetic anywhere in the oracle is reported by the sanitizers.  Besides running clean it checks
 * the few facts that hold whatever the field: the solves reach their residual, H_T is Hermitian on the driver's
 * vectors and H^{-1}(m, m) is the identity.  Exit status 0 on success.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

void or_gamma(int mu, cplx *out);
void or_hop(const int *L, int tbc, const cplx *U, const cplx *in, cplx *out, int dag);
void or_dw(const int *L, int tbc, double m0, const cplx *U, const cplx *in, cplx *out, int dag);
int or_mpm(int Ns, const double *omega, double m, int chir, double *M);
int or_k_omega(int Ns, const double *omega, double mj, double mi, int chir, double *k, double *Om, double *rem);
int or_dt(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm, const cplx *U,
          const cplx *in, cplx *out, int dag);
int or_ht(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm, const cplx *U,
          const cplx *in, cplx *out);
void or_dodwf(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm, const cplx *U,
              const cplx *in, cplx *out, int dag);
int or_ht_solve(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm, const cplx *U,
                const cplx *b, cplx *x, double tol, int maxit, double *relres);
int or_dodwf_solve(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
                   const cplx *U, const cplx *bp, cplx *y, double tol, int maxit, double *relres);
int or_chiral_action(const int *L, int tbc, double m0, int Ns, const double *omega, int chir, double m3, double m4,
                     double mo, const cplx *U, const cplx *phi, cplx *out, double tol, int maxit, double *S,
                     double *Sim, double *relres);
int or_hinv(const int *L, int tbc, double m0, int Ns, const double *omega, double mlo, double mhi, const cplx *U,
            const cplx *phi, cplx *out, double tol, int maxit, double *S, double *Sim, double *relres2);
int or_num_threads(void);
int or_at_inv(const int *L, double m0, int Ns, const double *omega, double mp, double mm, const cplx *in,
              cplx *out, int par, int dag);
int or_schur(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm, const cplx *U,
             const cplx *in, cplx *out, int dag);
int or_dt_at(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm, const cplx *U,
             const cplx *in, long nsites, const long *sites, cplx *out, int dag);

static unsigned long long rng_state = 88172645463325252ULL;

static double uniform(void)   /* xorshift64, (0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return ((rng_state >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

static cplx gauss(void)
{
    double r = sqrt(-log(uniform())), a = 6.283185307179586 * uniform();
    return r * cos(a) + I * r * sin(a);
}

/* a unitary 3x3 matrix with det 1: Gram-Schmidt on two random rows, the third their conjugate cross product */
static void random_su3(cplx *u)
{
    cplx a[3], b[3];
    for (int i = 0; i < 3; i++) { a[i] = gauss(); b[i] = gauss(); }
    double na = 0;
    for (int i = 0; i < 3; i++) na += creal(a[i] * conj(a[i]));
    for (int i = 0; i < 3; i++) a[i] /= sqrt(na);
    cplx d = 0;
    for (int i = 0; i < 3; i++) d += conj(a[i]) * b[i];
    double nb = 0;
    for (int i = 0; i < 3; i++) { b[i] -= d * a[i]; nb += creal(b[i] * conj(b[i])); }
    for (int i = 0; i < 3; i++) b[i] /= sqrt(nb);
    for (int i = 0; i < 3; i++) { u[i] = a[i]; u[3 + i] = b[i]; }
    u[6] = conj(a[1] * b[2] - a[2] * b[1]);
    u[7] = conj(a[2] * b[0] - a[0] * b[2]);
    u[8] = conj(a[0] * b[1] - a[1] * b[0]);
}

static int failures = 0;

static void check(int ok, const char *what, int Ns)
{
    if (!ok) {
        fprintf(stderr, "FAIL Ns=%d: %s\n", Ns, what);
        failures++;
    }
}

static cplx dot(long n, const cplx *a, const cplx *b)
{
    cplx s = 0;
    for (long i = 0; i < n; i++) s += conj(a[i]) * b[i];
    return s;
}

static void run(const int *L, int Ns)
{
    const double m0 = 1.3, tol = 1e-10;
    const int tbc = -1, maxit = 4000;
    long V = (long)L[0] * L[1] * L[2] * L[3], n4 = V * 12, n5 = n4 * Ns;
    double *om = malloc(sizeof(double) * Ns), *M = malloc(sizeof(double) * Ns * Ns), *Om = malloc(sizeof(double) * Ns);
    for (int s = 0; s < Ns; s++) {   /* positive and symmetric under s -> Ns - 1 - s */
        int d = s < Ns - 1 - s ? s : Ns - 1 - s;
        om[s] = 0.4 + 0.3 * d;
    }
    cplx *U = malloc(sizeof(cplx) * V * 4 * 9);
    for (long i = 0; i < V * 4; i++) random_su3(U + 9 * i);
    cplx *a = malloc(sizeof(cplx) * n5), *b = malloc(sizeof(cplx) * n5), *c = malloc(sizeof(cplx) * n5);
    cplx *d = malloc(sizeof(cplx) * n5);
    for (long i = 0; i < n5; i++) { a[i] = gauss(); b[i] = gauss(); }

    cplx g[16];
    for (int mu = 0; mu < 5; mu++) or_gamma(mu, g);
    for (int dag = 0; dag < 2; dag++) {
        or_hop(L, tbc, U, a, c, dag);
        or_dw(L, tbc, m0, U, a, c, dag);
        check(or_dt(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, c, dag) == 0, "dt", Ns);
        or_dodwf(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, c, dag);
        check(or_schur(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, c, dag) == 0, "schur", Ns);
        for (int par = -1; par < 2; par++)
            check(or_at_inv(L, m0, Ns, om, 0.1, 0.3, a, c, par, dag) == 0, "at_inv", Ns);
        long sites[3] = {0, V / 2 + 1, V - 1};
        check(or_dt_at(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, 3, sites, c, dag) == 0, "dt_at", Ns);
    }
    for (int chir = -1; chir <= 1; chir += 2) {
        double k, rem;
        check(or_mpm(Ns, om, 0.05, chir, M) == 0, "mpm", Ns);
        check(or_k_omega(Ns, om, 0.05, 0.3, chir, &k, Om, &rem) == 0 && rem < 1e-10, "k_omega rank one", Ns);
        check(or_k_omega(Ns, om, 0.3, 0.3, chir, &k, Om, &rem) == 0 && k == 0.0, "k_omega equal masses", Ns);
    }
    /* H_T Hermitian: <a, H b> = <H a, b> */
    check(or_ht(L, tbc, m0, Ns, om, 0.1, 0.3, U, b, c) == 0 && or_ht(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, d) == 0,
          "ht", Ns);
    cplx l = dot(n5, a, c), r = dot(n5, d, b);
    check(cabs(l - r) <= 1e-12 * cabs(l), "ht hermitian", Ns);

    double rr, rr2[2], S, Sim;
    int it = or_ht_solve(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, c, tol, maxit, &rr);
    check(it > 0 && rr <= tol, "ht_solve", Ns);
    it = or_dodwf_solve(L, tbc, m0, Ns, om, 0.1, 0.3, U, a, c, tol, maxit, &rr);
    check(it > 0 && rr <= tol, "dodwf_solve", Ns);
    check(or_chiral_action(L, tbc, m0, Ns, om, -1, 1.0, 0.3, 1.0, U, a, c, tol, maxit, &S, &Sim, &rr) >= 0 && S > 0,
          "chiral_action -", Ns);
    check(or_chiral_action(L, tbc, m0, Ns, om, +1, 0.05, 0.3, 1.0, U, a, c, tol, maxit, &S, &Sim, &rr) >= 0 && S > 0,
          "chiral_action +", Ns);
    check(or_hinv(L, tbc, m0, Ns, om, 0.05, 0.3, U, a, c, tol, maxit, &S, &Sim, rr2) >= 0 && S > 0, "hinv", Ns);
    /* H^{-1}(m, m) = 1 */
    check(or_hinv(L, tbc, m0, Ns, om, 0.3, 0.3, U, a, c, tol, maxit, &S, &Sim, rr2) >= 0, "hinv equal", Ns);
    double e = 0, nrm = 0;
    for (long i = 0; i < n4; i++) { e += cabs(c[i] - a[i]); nrm += cabs(a[i]); }
    check(e <= 1e-13 * nrm, "hinv equal masses is the identity", Ns);
    /* a solve stopped by its iteration limit reports failure and stays in bounds */
    check(or_ht_solve(L, tbc, m0, Ns, om, 0.01, 0.01, U, a, c, 1e-14, 2, &rr) < 0, "ht_solve maxit", Ns);

    free(om); free(M); free(Om); free(U); free(a); free(b); free(c); free(d);
}

int main(void)
{
    const int L1[4] = {4, 2, 2, 4}, L2[4] = {2, 4, 2, 2};
    int nt = or_num_threads();
    run(L1, 4);
    run(L1, 5);
    run(L2, 8);
    printf("oracle sanitizer driver: %d thread(s), %d failure(s)\n", nt, failures);
    return failures != 0;
}
