/*
 * FP64 CPU oracle for the optimal domain-wall (ODWF) operators and the exact
 * one-flavour action (EOFA) of Chen & Chiu, "Mass preconditioning for the exact
 * one-flavor action in lattice QCD with domain-wall fermion".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; it exists so that the HIP library can be checked against a plain,
 * slow, obviously correct implementation written from the definitions.  It
 * shares no code, header or table with the HIP path.
 *
 * Conventions (the paper defers the operator definitions to its references;
 * the readings used here are listed with each function):
 *   - site index lex = x + Lx*(y + Ly*(z + Lz*t)), mu = 0..3 is x,y,z,t;
 *   - links U[lex][mu][a][b] (row a, column b), complex128;
 *   - 4D spinor psi[lex][spin][colour]; 5D spinor psi[s][lex][spin][colour];
 *   - chiral gamma basis: gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *     gamma_4 = [[0,1],[1,0]]; gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 is
 *     built here by matrix products; P_pm = (1 pm gamma_5)/2;
 *   - fermion boundary: periodic in x,y,z, phase t_bc across the t boundary.
 *
 * Everything is plain loops in double complex; the only parallelism is an
 * OpenMP loop over 4D sites.  Every function states the passage it follows.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static cplx G[5][4][4];       /* gamma_1..gamma_4 in G[0..3], gamma_5 in G[4] */
static int g_ready = 0;

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx c[4][4])
{
    cplx t[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += a[i][k] * b[k][j];
            t[i][j] = s;
        }
    memcpy(c, t, sizeof(t));
}

static void gamma_init(void)
{
    if (g_ready) return;
    /* Pauli matrices */
    cplx sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    memset(G, 0, sizeof(G));
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                G[k][a][2 + b] = -I * sig[k][a][b];
                G[k][2 + a][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 2; a++) { G[3][a][2 + a] = 1; G[3][2 + a][a] = 1; }
    cplx t[4][4];
    mat4_mul(G[0], G[1], t);
    mat4_mul(t, G[2], t);
    mat4_mul(t, G[3], G[4]);
    g_ready = 1;
}

/* returns gamma_mu (mu = 0..3) or gamma_5 (mu = 4), row-major 4x4, for tests */
void or_gamma(int mu, double complex *out)
{
    gamma_init();
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) out[4 * i + j] = G[mu][i][j];
}

static inline long lexi(const int *L, int x, int y, int z, int t)
{
    return x + (long)L[0] * (y + (long)L[1] * (z + (long)L[2] * t));
}

static inline void coords(const int *L, long i, int *c)
{
    c[0] = (int)(i % L[0]); i /= L[0];
    c[1] = (int)(i % L[1]); i /= L[1];
    c[2] = (int)(i % L[2]); i /= L[2];
    c[3] = (int)i;
}

/* spin matrix (1 + sgn*gamma_mu) applied to a spinor chi[4][3] */
static inline void spin_proj(int mu, double sgn, const cplx chi[4][3], cplx out[4][3])
{
    for (int a = 0; a < 4; a++)
        for (int c = 0; c < 3; c++) {
            cplx s = chi[a][c];
            for (int b = 0; b < 4; b++)
                if (G[mu][a][b] != 0) s += sgn * G[mu][a][b] * chi[b][c];
            out[a][c] = s;
        }
}

/*
 * Wilson hopping term at one site (the sigma.t and W parts of the chiral block
 * form in Eq.(DTm1m2), written with links):
 *   hop psi(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                       + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ].
 * dag != 0 gives the adjoint hop (1 - gamma) <-> (1 + gamma), i.e. gamma_5 hop gamma_5.
 */
static void hop_site(const int *L, int tbc, const cplx *U, const cplx *in, long i, int dag,
                     cplx out[4][3])
{
    int c[4];
    coords(L, i, c);
    memset(out, 0, sizeof(cplx) * 12);
    for (int mu = 0; mu < 4; mu++) {
        int f[4] = {c[0], c[1], c[2], c[3]}, b[4] = {c[0], c[1], c[2], c[3]};
        f[mu] = (c[mu] + 1) % L[mu];
        b[mu] = (c[mu] - 1 + L[mu]) % L[mu];
        double phf = (mu == 3 && c[3] == L[3] - 1) ? (double)tbc : 1.0;
        double phb = (mu == 3 && c[3] == 0) ? (double)tbc : 1.0;
        long jf = lexi(L, f[0], f[1], f[2], f[3]);
        long jb = lexi(L, b[0], b[1], b[2], b[3]);
        const cplx *Uf = U + (i * 4 + mu) * 9;   /* U_mu(x)    */
        const cplx *Ub = U + (jb * 4 + mu) * 9;  /* U_mu(x-mu) */
        cplx chi[4][3], pr[4][3];
        /* forward: U_mu(x) psi(x+mu) */
        for (int a = 0; a < 4; a++)
            for (int r = 0; r < 3; r++) {
                cplx s = 0;
                for (int k = 0; k < 3; k++) s += Uf[3 * r + k] * in[(jf * 4 + a) * 3 + k];
                chi[a][r] = phf * s;
            }
        spin_proj(mu, dag ? +1.0 : -1.0, (const cplx(*)[3])chi, pr);
        for (int a = 0; a < 4; a++)
            for (int r = 0; r < 3; r++) out[a][r] += pr[a][r];
        /* backward: U_mu(x-mu)^dagger psi(x-mu) */
        for (int a = 0; a < 4; a++)
            for (int r = 0; r < 3; r++) {
                cplx s = 0;
                for (int k = 0; k < 3; k++) s += conj(Ub[3 * k + r]) * in[(jb * 4 + a) * 3 + k];
                chi[a][r] = phb * s;
            }
        spin_proj(mu, dag ? -1.0 : +1.0, (const cplx(*)[3])chi, pr);
        for (int a = 0; a < 4; a++)
            for (int r = 0; r < 3; r++) out[a][r] += pr[a][r];
    }
}

/* out = hop(in) on a 4D field (see hop_site) */
void or_hop(const int *L, int tbc, const double complex *U, const double complex *in,
            double complex *out, int dag)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx o[4][3];
        hop_site(L, tbc, U, in, i, dag, o);
        memcpy(out + i * 12, o, sizeof(o));
    }
}

/*
 * 4D Wilson operator with negative mass -m0 (the W - m0 + sigma.t of Eq.(DTm1m2)):
 *   D_w = (4 - m0) - hop/2;  dag != 0 gives D_w^dagger.
 */
void or_dw(const int *L, int tbc, double m0, const double complex *U, const double complex *in,
           double complex *out, int dag)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx o[4][3];
        hop_site(L, tbc, U, in, i, dag, o);
        for (int a = 0; a < 12; a++) out[i * 12 + a] = (4.0 - m0) * in[i * 12 + a] - 0.5 * ((cplx *)o)[a];
    }
}

/* ---------------------------------------------------------------- s-space */

/* L_+(m): (L_+)_{s,s-1} = 1, (L_+)_{1,Ns} = -m; L_-(m) = L_+(m)^T. Row-major Ns x Ns. */
static void lmat(int Ns, double m, int chir, double *Lm)
{
    memset(Lm, 0, sizeof(double) * Ns * Ns);
    for (int s = 1; s < Ns; s++) Lm[s * Ns + (s - 1)] = 1.0;
    Lm[0 * Ns + (Ns - 1)] = -m;
    if (chir < 0) {
        for (int i = 0; i < Ns; i++)
            for (int j = i + 1; j < Ns; j++) {
                double t = Lm[i * Ns + j];
                Lm[i * Ns + j] = Lm[j * Ns + i];
                Lm[j * Ns + i] = t;
            }
    }
}

/* Gauss-Jordan inverse with partial pivoting of a dense real n x n matrix. Returns 0 on success. */
static int invert(int n, const double *A, double *Ainv)
{
    double *a = malloc(sizeof(double) * n * 2 * n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++) a[i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i);
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(a[r * 2 * n + col]) > fabs(a[piv * 2 * n + col])) piv = r;
        if (a[piv * 2 * n + col] == 0.0) { free(a); return -1; }
        if (piv != col)
            for (int j = 0; j < 2 * n; j++) {
                double t = a[col * 2 * n + j];
                a[col * 2 * n + j] = a[piv * 2 * n + j];
                a[piv * 2 * n + j] = t;
            }
        double d = a[col * 2 * n + col];
        for (int j = 0; j < 2 * n; j++) a[col * 2 * n + j] /= d;
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            double f = a[r * 2 * n + col];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; j++) a[r * 2 * n + j] -= f * a[col * 2 * n + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = a[i * 2 * n + n + j];
    free(a);
    return 0;
}

/*
 * M_pm(m) = omega^{-1/2} (1 - L_pm(m)) (1 + L_pm(m))^{-1} omega^{-1/2}, the s-space
 * blocks of Eq.(DTm1m2) for the optimal DWF with rho_s = sigma_s = omega_s (the
 * reading under which m_PV = 2 m0 as in Sec. III).  chir = +1 or -1.
 */
int or_mpm(int Ns, const double *omega, double m, int chir, double *M)
{
    double *Lm = malloc(sizeof(double) * Ns * Ns), *A = malloc(sizeof(double) * Ns * Ns);
    double *Ai = malloc(sizeof(double) * Ns * Ns);
    lmat(Ns, m, chir, Lm);
    for (int i = 0; i < Ns; i++)
        for (int j = 0; j < Ns; j++) A[i * Ns + j] = (i == j) + Lm[i * Ns + j];
    int rc = invert(Ns, A, Ai);
    for (int i = 0; i < Ns; i++)
        for (int j = 0; j < Ns; j++) {
            double s = 0;
            for (int k = 0; k < Ns; k++) s += ((i == k) - Lm[i * Ns + k]) * Ai[k * Ns + j];
            M[i * Ns + j] = s / sqrt(omega[i] * omega[j]);
        }
    free(Lm); free(A); free(Ai);
    return rc;
}

/*
 * Rank-one mass difference of Eq.(delta_ij): Delta_pm(mj, mi) = R5 (M_pm(mj) - M_pm(mi)).
 * The oracle does not use the closed form of Eq.(k_ij) (its constants c and lambda
 * are not defined in the paper); it forms the dense difference and factors it as
 * Delta = k * Om Om^T with Om = the column of Delta with the largest diagonal entry
 * and k = 1 / Delta_cc.  Returns the relative size of the rank-one remainder in *rem.
 */
int or_k_omega(int Ns, const double *omega, double mj, double mi, int chir, double *k, double *Om,
               double *rem)
{
    double *Mj = malloc(sizeof(double) * Ns * Ns), *Mi = malloc(sizeof(double) * Ns * Ns);
    double *D = malloc(sizeof(double) * Ns * Ns);
    int rc = or_mpm(Ns, omega, mj, chir, Mj) | or_mpm(Ns, omega, mi, chir, Mi);
    for (int i = 0; i < Ns; i++)
        for (int j = 0; j < Ns; j++)
            D[i * Ns + j] = Mj[(Ns - 1 - i) * Ns + j] - Mi[(Ns - 1 - i) * Ns + j];
    int c = 0;
    for (int i = 1; i < Ns; i++)
        if (fabs(D[i * Ns + i]) > fabs(D[c * Ns + c])) c = i;
    double dcc = D[c * Ns + c];
    if (dcc == 0.0) {
        *k = 0.0;
        for (int i = 0; i < Ns; i++) Om[i] = 0.0;
        *rem = 0.0;
    } else {
        for (int i = 0; i < Ns; i++) Om[i] = D[i * Ns + c];
        *k = 1.0 / dcc;
        double num = 0, den = 0;
        for (int i = 0; i < Ns; i++)
            for (int j = 0; j < Ns; j++) {
                double r = D[i * Ns + j] - (*k) * Om[i] * Om[j];
                num += r * r;
                den += D[i * Ns + j] * D[i * Ns + j];
            }
        *rem = sqrt(num / den);
    }
    free(Mj); free(Mi); free(D);
    return rc;
}

/* chiral projector coefficient: (P_chir)_{ab} from gamma_5 */
static inline cplx pch(int chir, int a, int b)
{
    return 0.5 * ((a == b) + chir * G[4][a][b]);
}

/*
 * D_T(m+, m-) = D_w + P_+ M_+(m+) + P_- M_-(m-) on a 5D field (Eq.(DTm1m2)).
 * dag != 0: D_T^dagger = D_w^dagger + P_+ M_+^T + P_- M_-^T.
 */
int or_dt(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
          const double complex *U, const double complex *in, double complex *out, int dag)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    double *Mp = malloc(sizeof(double) * Ns * Ns), *Mm = malloc(sizeof(double) * Ns * Ns);
    int rc = or_mpm(Ns, omega, mp, +1, Mp) | or_mpm(Ns, omega, mm, -1, Mm);
    for (int s = 0; s < Ns; s++) or_dw(L, tbc, m0, U, in + s * V * 12, out + s * V * 12, dag);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        for (int s = 0; s < Ns; s++) {
            cplx acc[12] = {0};
            for (int t = 0; t < Ns; t++) {
                double cp = dag ? Mp[t * Ns + s] : Mp[s * Ns + t];
                double cm = dag ? Mm[t * Ns + s] : Mm[s * Ns + t];
                const cplx *src = in + (t * V + i) * 12;
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx p = cp * pch(+1, a, b) + cm * pch(-1, a, b);
                        if (p == 0) continue;
                        for (int c = 0; c < 3; c++) acc[a * 3 + c] += p * src[b * 3 + c];
                    }
            }
            for (int a = 0; a < 12; a++) out[(s * V + i) * 12 + a] += acc[a];
        }
    }
    free(Mp); free(Mm);
    return rc;
}

/* H_T(m+, m-) = gamma_5 R5 D_T(m+, m-)  (the Hermitian operator of Eq.(H)), (R5 psi)_s = psi_{Ns+1-s} */
int or_ht(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
          const double complex *U, const double complex *in, double complex *out)
{
    long V = (long)L[0] * L[1] * L[2] * L[3];
    cplx *tmp = malloc(sizeof(cplx) * V * 12 * Ns);
    int rc = or_dt(L, tbc, m0, Ns, omega, mp, mm, U, in, tmp, 0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++)
        for (int s = 0; s < Ns; s++)
            for (int a = 0; a < 4; a++)
                for (int c = 0; c < 3; c++) {
                    cplx v = 0;
                    for (int b = 0; b < 4; b++) v += G[4][a][b] * tmp[((Ns - 1 - s) * V + i) * 12 + b * 3 + c];
                    out[(s * V + i) * 12 + a * 3 + c] = v;
                }
    free(tmp);
    return rc;
}

/* (1 + sgn*L) psi with L = P_+ L_+(m+) + P_- L_-(m-); transp != 0 uses L^T. */
static void one_pm_l(int Ns, long V, double mp, double mm, double sgn, int transp, const cplx *in,
                     cplx *out)
{
    double *Lp = malloc(sizeof(double) * Ns * Ns), *Lm = malloc(sizeof(double) * Ns * Ns);
    lmat(Ns, mp, +1, Lp);
    lmat(Ns, mm, -1, Lm);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++)
        for (int s = 0; s < Ns; s++)
            for (int a = 0; a < 4; a++)
                for (int c = 0; c < 3; c++) {
                    cplx v = in[(s * V + i) * 12 + a * 3 + c];
                    for (int t = 0; t < Ns; t++) {
                        double lp = transp ? Lp[t * Ns + s] : Lp[s * Ns + t];
                        double lm = transp ? Lm[t * Ns + s] : Lm[s * Ns + t];
                        if (lp == 0 && lm == 0) continue;
                        for (int b = 0; b < 4; b++) {
                            cplx p = lp * pch(+1, a, b) + lm * pch(-1, a, b);
                            if (p != 0) v += sgn * p * in[(t * V + i) * 12 + b * 3 + c];
                        }
                    }
                    out[(s * V + i) * 12 + a * 3 + c] = v;
                }
    free(Lp); free(Lm);
}

/*
 * Optimal DWF operator (the D(m) of Eq.(detDodwf)) in the reading
 *   D_odwf(m+, m-) = D_w omega (1 + L) + (1 - L),   L = P_+ L_+(m+) + P_- L_-(m-),
 * so that D_T = omega^{-1/2} D_odwf (1 + L)^{-1} omega^{-1/2}.
 * dag != 0: D_odwf^dagger = (1 + L)^T omega D_w^dagger + (1 - L)^T.
 */
void or_dodwf(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
              const double complex *U, const double complex *in, double complex *out, int dag)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    long n = V * 12;
    cplx *a = malloc(sizeof(cplx) * n * Ns), *b = malloc(sizeof(cplx) * n * Ns);
    if (!dag) {
        one_pm_l(Ns, V, mp, mm, +1.0, 0, in, a);                        /* (1+L) in        */
        for (int s = 0; s < Ns; s++)
            for (long j = 0; j < n; j++) a[s * n + j] *= omega[s];          /* omega (1+L) in  */
        for (int s = 0; s < Ns; s++) or_dw(L, tbc, m0, U, a + s * n, out + s * n, 0);
        one_pm_l(Ns, V, mp, mm, -1.0, 0, in, b);                        /* (1-L) in        */
    } else {
        for (int s = 0; s < Ns; s++) or_dw(L, tbc, m0, U, in + s * n, a + s * n, 1);
        for (int s = 0; s < Ns; s++)
            for (long j = 0; j < n; j++) a[s * n + j] *= omega[s];
        one_pm_l(Ns, V, mp, mm, +1.0, 1, a, out);                       /* (1+L)^T omega Dw^+ */
        one_pm_l(Ns, V, mp, mm, -1.0, 1, in, b);                        /* (1-L)^T in      */
    }
    for (long j = 0; j < n * Ns; j++) out[j] += b[j];
    free(a); free(b);
}

static double nrm2(long n, const cplx *v)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s)
    for (long i = 0; i < n; i++) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return s;
}

/*
 * Solve H_T(m+, m-) x = b (5D), the inverse inside Eqs.(Hij), (m1m2_m1m4) and (m1m2_m3m2).
 * H_T is Hermitian, so the plain route is CG on the normal equations H_T^2 x = H_T b (the
 * CG of the force and heat-bath solves of Sec. I), over the full lattice, without
 * preconditioning.  Stops when the recomputed true residual ||b - H_T x|| / ||b|| <= tol / 10
 * and reports it in *relres.  Returns the number of CG iterations, or -1 if maxit was reached.
 */
int or_ht_solve(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
                const double complex *U, const double complex *b, double complex *x, double tol,
                int maxit, double *relres)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    long n = V * 12 * Ns;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    memset(x, 0, sizeof(cplx) * n);
    double bn2 = nrm2(n, b);
    int it = 0, fail = 0;
    for (;;) {
        /* true residual t = b - H_T x */
        or_ht(L, tbc, m0, Ns, omega, mp, mm, U, x, t);
        for (long j = 0; j < n; j++) t[j] = b[j] - t[j];
        *relres = sqrt(nrm2(n, t) / bn2);
        if (*relres <= 0.1 * tol || bn2 == 0.0) break;
        if (it >= maxit) { fail = 1; break; }
        /* (re)start: r = H_T t, p = r */
        or_ht(L, tbc, m0, Ns, omega, mp, mm, U, t, r);
        memcpy(p, r, sizeof(cplx) * n);
        double rr = nrm2(n, r), rr0 = rr;
        while (it < maxit) {
            or_ht(L, tbc, m0, Ns, omega, mp, mm, U, p, q);
            double alpha = rr / nrm2(n, q);
            or_ht(L, tbc, m0, Ns, omega, mp, mm, U, q, t);
            for (long j = 0; j < n; j++) { x[j] += alpha * p[j]; r[j] -= alpha * t[j]; }
            double rn = nrm2(n, r);
            it++;
            if (rn <= 1e-4 * tol * tol * rr0) break;   /* go back and check the true residual */
            double beta = rn / rr;
            for (long j = 0; j < n; j++) p[j] = r[j] + beta * p[j];
            rr = rn;
        }
    }
    free(r); free(p); free(q); free(t);
    return fail ? -1 : it;
}

/*
 * Solve D_odwf(m+, m-) y = b' by CGNR over the full lattice (no preconditioning); used to
 * check the route H_T^{-1} = omega^{1/2} (1 + L) D_odwf^{-1} omega^{1/2} R5 gamma_5 against
 * the direct H_T solve.  Returns iterations (or -1) and the D_odwf residual in *relres.
 */
int or_dodwf_solve(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
                   const double complex *U, const double complex *bp, double complex *y, double tol,
                   int maxit, double *relres)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    long n = V * 12 * Ns;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    memset(y, 0, sizeof(cplx) * n);
    double bn2 = nrm2(n, bp);
    int it = 0, fail = 0;
    for (;;) {
        or_dodwf(L, tbc, m0, Ns, omega, mp, mm, U, y, t, 0);
        for (long j = 0; j < n; j++) t[j] = bp[j] - t[j];
        *relres = sqrt(nrm2(n, t) / bn2);
        if (*relres <= 0.1 * tol || bn2 == 0.0) break;
        if (it >= maxit) { fail = 1; break; }
        or_dodwf(L, tbc, m0, Ns, omega, mp, mm, U, t, r, 1);
        memcpy(p, r, sizeof(cplx) * n);
        double rr = nrm2(n, r), rr0 = rr;
        while (it < maxit) {
            or_dodwf(L, tbc, m0, Ns, omega, mp, mm, U, p, t, 0);
            double alpha = rr / nrm2(n, t);
            or_dodwf(L, tbc, m0, Ns, omega, mp, mm, U, t, q, 1);
            for (long j = 0; j < n; j++) { y[j] += alpha * p[j]; r[j] -= alpha * q[j]; }
            double rn = nrm2(n, r);
            it++;
            if (rn <= 1e-4 * tol * tol * rr0) break;
            double beta = rn / rr;
            for (long j = 0; j < n; j++) p[j] = r[j] + beta * p[j];
            rr = rn;
        }
    }
    free(r); free(p); free(q); free(t);
    return fail ? -1 : it;
}

/*
 * One chiral EOFA action, Eqs.(m1m2_m1m4) and (m1m2_m3m2):
 *   chir = -1: (m3,m4)/(m3,mo):  out = P_- [ phi - k(mo,m4) Om^T H_T(m3,m4)^{-1} Om P_- phi ]
 *   chir = +1: (m3,m4)/(mo,m4):  out = P_+ [ phi + k(mo,m3) Om^T H_T(m3,m4)^{-1} Om P_+ phi ]
 * where k Om Om^T is the dense rank-one Delta_chir of or_k_omega.  *S = Re phi^dag out,
 * *Sim its imaginary part.  Returns the CG iteration count (or -1).
 */
int or_chiral_action(const int *L, int tbc, double m0, int Ns, const double *omega, int chir,
                     double m3, double m4, double mo, const double complex *U,
                     const double complex *phi, double complex *out, double tol, int maxit,
                     double *S, double *Sim, double *relres)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    double *Om = malloc(sizeof(double) * Ns), k, rem;
    if (chir < 0) or_k_omega(Ns, omega, mo, m4, -1, &k, Om, &rem);
    else or_k_omega(Ns, omega, mo, m3, +1, &k, Om, &rem);
    cplx *pphi = malloc(sizeof(cplx) * V * 12), *b = malloc(sizeof(cplx) * V * 12 * Ns);
    cplx *x = malloc(sizeof(cplx) * V * 12 * Ns);
    for (long i = 0; i < V; i++)
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx v = 0;
                for (int bb = 0; bb < 4; bb++) v += pch(chir, a, bb) * phi[i * 12 + bb * 3 + c];
                pphi[i * 12 + a * 3 + c] = v;
            }
    for (int s = 0; s < Ns; s++)
        for (long j = 0; j < V * 12; j++) b[s * V * 12 + j] = Om[s] * pphi[j];
    int it = or_ht_solve(L, tbc, m0, Ns, omega, m3, m4, U, b, x, tol, maxit, relres);
    cplx sacc = 0;
    for (long i = 0; i < V; i++)
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx proj = 0;
                for (int s = 0; s < Ns; s++) {
                    cplx v = 0;
                    for (int bb = 0; bb < 4; bb++) v += pch(chir, a, bb) * x[(s * V + i) * 12 + bb * 3 + c];
                    proj += Om[s] * v;
                }
                cplx o = pphi[i * 12 + a * 3 + c] + (double)chir * k * proj;
                out[i * 12 + a * 3 + c] = o;
                sacc += conj(phi[i * 12 + a * 3 + c]) * o;
            }
    *S = creal(sacc);
    *Sim = cimag(sacc);
    free(Om); free(pphi); free(b); free(x);
    return it;
}

/*
 * H^{-1}(mj, mi) phi of Eq.(Hij) as the sum of its two chiral parts (Eq.(pfij)):
 *   - part (mi,mi)/(mi,mj) and + part (mi,mj)/(mj,mj).
 * (H_T(mj) - Delta_+(mj,mi) P_+ = H_T(mi,mj), so the + part is Eq.(m1m2_m3m2) with m3 = mi,
 *  m4 = mj, m1 = mj.)  *S = phi^dag H^{-1} phi.
 */
int or_hinv(const int *L, int tbc, double m0, int Ns, const double *omega, double mlo, double mhi,
            const double complex *U, const double complex *phi, double complex *out, double tol,
            int maxit, double *S, double *Sim, double *relres2)
{
    long V = (long)L[0] * L[1] * L[2] * L[3];
    cplx *o2 = malloc(sizeof(cplx) * V * 12);
    double s1, s1i, s2, s2i;
    int i1 = or_chiral_action(L, tbc, m0, Ns, omega, -1, mlo, mlo, mhi, U, phi, out, tol, maxit, &s1,
                              &s1i, &relres2[0]);
    int i2 = or_chiral_action(L, tbc, m0, Ns, omega, +1, mlo, mhi, mhi, U, phi, o2, tol, maxit, &s2,
                              &s2i, &relres2[1]);
    for (long j = 0; j < V * 12; j++) out[j] += o2[j];
    *S = s1 + s2;
    *Sim = s1i + s2i;
    free(o2);
    return (i1 < 0 || i2 < 0) ? -1 : i1 + i2;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------- even-odd (test support) */

/*
 * Site-local block of D_T: A_T = (4 - m0) + P_+ M_+(m+) + P_- M_-(m-) (the diagonal
 * in x of Eq.(DTm1m2)).  out = A_T^{-1} in (dag: A_T^{-dagger} in) on the 4D sites
 * whose parity equals par (par = -1: all sites); other sites of out are set to zero.
 * The inverse is a dense Gauss-Jordan inverse per chirality.
 */
int or_at_inv(const int *L, double m0, int Ns, const double *omega, double mp, double mm,
              const double complex *in, double complex *out, int par, int dag)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    double *Mp = malloc(sizeof(double) * Ns * Ns), *Mm = malloc(sizeof(double) * Ns * Ns);
    double *Ip = malloc(sizeof(double) * Ns * Ns), *Im = malloc(sizeof(double) * Ns * Ns);
    int rc = or_mpm(Ns, omega, mp, +1, Mp) | or_mpm(Ns, omega, mm, -1, Mm);
    for (int i = 0; i < Ns; i++) { Mp[i * Ns + i] += 4.0 - m0; Mm[i * Ns + i] += 4.0 - m0; }
    rc |= invert(Ns, Mp, Ip) | invert(Ns, Mm, Im);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        int c[4];
        coords(L, i, c);
        int keep = par < 0 || ((c[0] + c[1] + c[2] + c[3]) & 1) == par;
        for (int s = 0; s < Ns; s++)
            for (int a = 0; a < 4; a++)
                for (int cc = 0; cc < 3; cc++) {
                    cplx v = 0;
                    if (keep)
                        for (int t = 0; t < Ns; t++) {
                            double ap = dag ? Ip[t * Ns + s] : Ip[s * Ns + t];
                            double am = dag ? Im[t * Ns + s] : Im[s * Ns + t];
                            for (int b = 0; b < 4; b++) {
                                cplx p = ap * pch(+1, a, b) + am * pch(-1, a, b);
                                if (p != 0) v += p * in[(t * V + i) * 12 + b * 3 + cc];
                            }
                        }
                    out[(s * V + i) * 12 + a * 3 + cc] = v;
                }
    }
    free(Mp); free(Mm); free(Ip); free(Im);
    return rc;
}

static void keep_parity(const int *L, int Ns, cplx *f, int par)
{
    long V = (long)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        int c[4];
        coords(L, i, c);
        if (((c[0] + c[1] + c[2] + c[3]) & 1) != par)
            for (int s = 0; s < Ns; s++) memset(f + (s * V + i) * 12, 0, sizeof(cplx) * 12);
    }
}

/*
 * Schur complement of D_T on the odd sites, normalised by the site-local block:
 *   Dhat = 1 - A_T^{-1} (D_T)_{oe} A_T^{-1} (D_T)_{eo}     (dag: its adjoint),
 * built from the oracle's own D_T blocks.  in/out are full 5D fields; only odd sites
 * of in are read and only odd sites of out are non-zero.  (Even-odd preconditioning
 * is not in the paper; this is the textbook Schur complement of the 2x2 parity blocks.)
 */
int or_schur(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
             const double complex *U, const double complex *in, double complex *out, int dag)
{
    long V = (long)L[0] * L[1] * L[2] * L[3];
    long n = V * 12 * Ns;
    cplx *a = malloc(sizeof(cplx) * n), *b = malloc(sizeof(cplx) * n);
    int rc = 0;
    memcpy(a, in, sizeof(cplx) * n);
    keep_parity(L, Ns, a, 1);
    if (!dag) {
        rc |= or_dt(L, tbc, m0, Ns, omega, mp, mm, U, a, b, 0);
        keep_parity(L, Ns, b, 0);                                /* (D_T)_eo x_o */
        rc |= or_at_inv(L, m0, Ns, omega, mp, mm, b, a, 0, 0);
        rc |= or_dt(L, tbc, m0, Ns, omega, mp, mm, U, a, b, 0);
        keep_parity(L, Ns, b, 1);                                /* (D_T)_oe ... */
        rc |= or_at_inv(L, m0, Ns, omega, mp, mm, b, a, 1, 0);
    } else {
        rc |= or_at_inv(L, m0, Ns, omega, mp, mm, a, b, 1, 1);
        rc |= or_dt(L, tbc, m0, Ns, omega, mp, mm, U, b, a, 1);
        keep_parity(L, Ns, a, 0);
        rc |= or_at_inv(L, m0, Ns, omega, mp, mm, a, b, 0, 1);
        rc |= or_dt(L, tbc, m0, Ns, omega, mp, mm, U, b, a, 1);
        keep_parity(L, Ns, a, 1);
    }
    for (long j = 0; j < n; j++) out[j] = in[j] - a[j];
    keep_parity(L, Ns, out, 1);
    free(a); free(b);
    return rc;
}

/*
 * D_T(m+, m-) (dag: D_T^dagger) evaluated only at the 4D sites listed in sites[]
 * (lexicographic indices), all s.  out[k][s][spin][colour].  For checks of very large
 * lattices where a full oracle application is too slow.
 */
int or_dt_at(const int *L, int tbc, double m0, int Ns, const double *omega, double mp, double mm,
             const double complex *U, const double complex *in, long nsites, const long *sites,
             double complex *out, int dag)
{
    gamma_init();
    long V = (long)L[0] * L[1] * L[2] * L[3];
    double *Mp = malloc(sizeof(double) * Ns * Ns), *Mm = malloc(sizeof(double) * Ns * Ns);
    int rc = or_mpm(Ns, omega, mp, +1, Mp) | or_mpm(Ns, omega, mm, -1, Mm);
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < nsites; k++) {
        long i = sites[k];
        for (int s = 0; s < Ns; s++) {
            cplx o[4][3];
            hop_site(L, tbc, U, in + (long)s * V * 12, i, dag, o);
            cplx *dst = out + (k * Ns + s) * 12;
            for (int a = 0; a < 12; a++) dst[a] = (4.0 - m0) * in[((long)s * V + i) * 12 + a] - 0.5 * ((cplx *)o)[a];
            for (int t = 0; t < Ns; t++) {
                double cp = dag ? Mp[t * Ns + s] : Mp[s * Ns + t];
                double cm = dag ? Mm[t * Ns + s] : Mm[s * Ns + t];
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx p = cp * pch(+1, a, b) + cm * pch(-1, a, b);
                        if (p == 0) continue;
                        for (int c = 0; c < 3; c++) dst[a * 3 + c] += p * in[((long)t * V + i) * 12 + b * 3 + c];
                    }
            }
        }
    }
    free(Mp); free(Mm);
    return rc;
}
