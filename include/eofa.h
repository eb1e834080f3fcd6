/*
 * eofa.h - C ABI of the MI355X (gfx950) EOFA / optimal domain-wall solver library.
 *
 * The library solves the 5D Hermitian systems H_T(m+, m-) x = b of the exact
 * one-flavour pseudofermion action (EOFA) and assembles, from their solutions,
 * H^{-1}(mj, mi) phi of Eq.(Hij) and the action S = phi^dagger H^{-1} phi
 * (Chen & Chiu, "Mass preconditioning for the exact one-flavor action in lattice
 * QCD with domain-wall fermion", Sec. I and Sec. II).
 *
 * Operators (the paper defers their definitions to its references; this is the
 * reading the library implements):
 *   D_w          = (4 - m0) - (1/2) sum_mu [(1 - gamma_mu) U_mu(x) delta_{x+mu}
 *                                          + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu}]
 *                  (the W - m0 + sigma.t blocks of Eq.(DTm1m2));
 *   D_T(m+, m-)  = D_w + P_+ M_+(m+) + P_- M_-(m-),  Eq.(DTm1m2), with
 *   M_pm(m)      = omega^{-1/2} (1 - L_pm(m)) (1 + L_pm(m))^{-1} omega^{-1/2},
 *                  (L_+)_{s,s-1} = 1, (L_+)_{1,Ns} = -m, L_- = L_+^T;
 *   H_T(m+, m-)  = gamma_5 R5 D_T(m+, m-)  (Hermitian; (R5 psi)_s = psi_{Ns+1-s});
 *   k(mj, mi)    = 2 (mj - mi) / ((1 + mj)(1 + mi)),  Om_s = (-1)^s omega_s^{-1/2}
 *                  (Eqs.(delta_ij)-(k_ij) for this operator: Delta = k Om Om^T).
 * Chiral basis: gamma_5 = diag(1, 1, -1, -1), P_pm = (1 pm gamma_5)/2, fermion
 * fields periodic in x, y, z and with phase t_bc across the t boundary.
 *
 * Memory.  Every field pointer is a DEVICE pointer owned by the caller; the
 * library never frees it.  Canonical layouts (complex128 = 2 doubles re, im):
 *   links  U[Lt][Lz][Ly][Lx][mu][3][3]   (mu = x, y, z, t; row, column)
 *   4D     phi[Lt][Lz][Ly][Lx][spin 4][colour 3]
 *   5D     psi[Ns][Lt][Lz][Ly][Lx][spin 4][colour 3]
 * All work is enqueued on the context's hipStream_t; calls that return a host
 * scalar (S, info) synchronise that stream before returning.
 *
 * Errors.  Every call returns an eofa_status; nothing aborts and no C++
 * exception crosses this boundary.  eofa_last_error() returns the context's
 * last message.  A context is not thread-safe: use one per stream.
 */
#ifndef EOFA_H
#define EOFA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eofa_ctx eofa_ctx;

typedef enum {
    EOFA_OK = 0,
    EOFA_EINVAL = -1,   /* bad argument (message says which), including a source with NaN/Inf */
    EOFA_ENOMEM = -2,   /* device allocation or workspace too small */
    EOFA_EHIP = -3,     /* a HIP runtime call failed */
    EOFA_ENOCONV = -4,  /* solver hit max_iter or broke down; best iterate returned */
    EOFA_ESTATE = -5,   /* call out of order (e.g. no gauge field set) */
    EOFA_ENOTIMPL = -6
} eofa_status;

typedef enum { EOFA_FP64 = 0, EOFA_MIXED_FP32 = 1, EOFA_MIXED_FP16 = 2 } eofa_precision;
typedef enum { EOFA_PC_NONE = 0, EOFA_PC_LEARNED = 1 } eofa_precond;

typedef struct {
    double tol;            /* target true relative residual ||b - H_T x|| / ||b|| of every 5D solve */
    int max_iter;          /* total inner iterations allowed per 5D solve */
    eofa_precision prec;   /* storage precision of the inner Krylov solver */
    eofa_precond pc;       /* EOFA_PC_LEARNED: flexible GCR with the learned preconditioner */
    double reliable_delta; /* mixed precision: reliable update when ||r|| drops by this factor (0: 0.1) */
    int use_graph;         /* capture blocks of check_every CG iterations in a hipGraph (once per buffer
                              set, cached in the context) and replay them; same arithmetic as eager */
    int check_every;       /* iterations between host convergence checks (0: automatic) */
} eofa_solve_params;

typedef struct {
    int iters;             /* inner Krylov iterations */
    int op_applies;        /* applications of the even-odd operator Dhat (or its adjoint) */
    int reliable_updates;  /* FP64 residual recomputations (restarts included) */
    int fell_back;         /* the learned-preconditioner or reduced-precision solve handed over to FP64 CG */
    double true_rel_resid; /* FP64 ||b - H_T x|| / ||b|| of the returned x */
    double seconds;        /* wall time of the solve */
} eofa_solve_info;

/* Operators for eofa_apply (all on canonical 5D fields unless noted). */
typedef enum {
    EOFA_OP_DW = 0,        /* D_w on every s-slice */
    EOFA_OP_HOP = 1,       /* Wilson hop sum_mu[(1-g)U psi(x+mu) + (1+g)U^dag psi(x-mu)] on every slice */
    EOFA_OP_DT = 2,        /* D_T(m+, m-) */
    EOFA_OP_DT_DAG = 3,    /* D_T(m+, m-)^dagger */
    EOFA_OP_HT = 4,        /* H_T(m+, m-) */
    EOFA_OP_AT_INV = 5,    /* (4 - m0 + P_+ M_+ + P_- M_-)^{-1}, site-local */
    EOFA_OP_SCHUR = 6,     /* Dhat = 1 - A^{-1}(D_T)_oe A^{-1}(D_T)_eo on odd sites (even sites of out = 0) */
    EOFA_OP_SCHUR_DAG = 7, /* Dhat^dagger */
    EOFA_OP_SCHUR_NORMAL = 8, /* Dhat^dagger Dhat */
    EOFA_OP_DODWF = 9,     /* D_odwf(m+, m-) = D_w omega (1 + L) + (1 - L), the optimal DWF operator (Sec. III.A) */
    EOFA_OP_DODWF_DAG = 10, /* D_odwf(m+, m-)^dagger */
    EOFA_OP_HOP_EO = 11,   /* Wilson hop from the odd to the even sites (odd sites of out = 0) */
    EOFA_OP_HOP_OE = 12    /* Wilson hop from the even to the odd sites (even sites of out = 0) */
} eofa_op;

/*
 * Create a context for an Lx x Ly x Lz x Lt lattice (dims[] = {Lx, Ly, Lz, Lt}, each even,
 * Lx*Ly*Lz*Lt/2 < 2^31) with Ns fifth-dimension slices (Ns a power of two, 2..64),
 * Wilson mass -m0 (0 < m0 < 2), weights omega_host[Ns] (host memory, > 0, R5-symmetric to
 * 1e-14 relative: the optimal weights of Sec. III), fermion phase t_bc = -1 or +1 across the
 * t boundary, and the hipStream_t all work goes to (NULL: the default stream).
 */
eofa_status eofa_create(eofa_ctx **out, const int dims[4], int Ns, double m0,
                        const double *omega_host, int t_bc, void *hip_stream);

/* Workspace the solves below need for nrhs simultaneous systems under params. */
eofa_status eofa_workspace_size(const eofa_ctx *ctx, const eofa_solve_params *params, int nrhs,
                                size_t *bytes);
/* Caller-owned device workspace (256-byte aligned).  Without one, the library allocates
 * its own on first use and frees it in eofa_destroy. */
eofa_status eofa_set_workspace(eofa_ctx *ctx, void *dev_ptr, size_t bytes);

/* Upload and pack the gauge field (device pointer, canonical layout).  Must precede solves. */
eofa_status eofa_set_gauge(eofa_ctx *ctx, const void *U);

/*
 * out = H^{-1}(m_hi, m_lo) phi of Eq.(Hij) (m_lo = m_i, m_hi = m_j, 0 < m_lo <= m_hi <= 1),
 * computed as the - action (m_lo,m_lo)/(m_lo,m_hi) plus the + action (m_lo,m_hi)/(m_hi,m_hi)
 * (Eq.(pfij), chiral split of Sec. I).  phi, out: 4D canonical device buffers (may not alias).
 * *S = Re phi^dagger out (S may be NULL).  info[0] is the - solve, info[1] the + solve.
 */
eofa_status eofa_hinv(eofa_ctx *ctx, double m_lo, double m_hi, const void *phi, void *out, double *S,
                      const eofa_solve_params *params, eofa_solve_info info[2]);

/*
 * One chiral action of Eqs.(m1m2_m1m4) / (m1m2_m3m2):
 *   chir = -1: (m3,m4)/(m3,mo): out = P_- [phi - k(mo,m4) Om^T H_T(m3,m4)^{-1} Om P_- phi]
 *   chir = +1: (m3,m4)/(mo,m4): out = P_+ [phi + k(mo,m3) Om^T H_T(m3,m4)^{-1} Om P_+ phi]
 * phi, out: 4D canonical device buffers.  *S = Re phi^dagger out (may be NULL).
 */
eofa_status eofa_chiral_action(eofa_ctx *ctx, int chir, double m3, double m4, double mo,
                               const void *phi, void *out, double *S,
                               const eofa_solve_params *params, eofa_solve_info *info);

/*
 * Fermion force of one chiral action (the molecular-dynamics derivative of S above; the force of a
 * pseudofermion action enters the HMC of Sec. I, and each factor of the splittings of Sec. II has its own):
 *   force[mu][site][a] = dS/dw^a  for  U_mu(site) -> exp(i w^a T^a) U_mu(site),  T^a = lambda^a / 2,
 * with mu = 0..3 for x, y, z, t and the site in canonical order (x fastest).  Equals -c k x^dag (dH_T/dw^a) x
 * with x = H_T(m3,m4)^{-1} Om P_c phi and c = chir.  phi: 4D canonical device buffer; force: caller-owned
 * device buffer of 4 * V * 8 doubles.  *S as for eofa_chiral_action (may be NULL).  Solves as
 * eofa_chiral_action does (same params); EOFA_ENOCONV still writes the force of the last iterate.
 */
eofa_status eofa_chiral_force(eofa_ctx *ctx, int chir, double m3, double m4, double mo, const void *phi,
                              double *force, double *S, const eofa_solve_params *params, eofa_solve_info *info);

/*
 * n independent chiral actions solved together (the multi-RHS form): action j has chirality
 * chir[j] and masses (m3[j], m4[j], mo[j]) as in eofa_chiral_action, source phi[j] and output
 * out[j] (arrays of n device pointers held in HOST memory).  S[j] (host, may be NULL), info[j].
 * Up to 8 systems go through each launch sequence, each with its own masses; links are loaded
 * once per site for the whole group.
 */
eofa_status eofa_chiral_action_batch(eofa_ctx *ctx, int n, const int *chir, const double *m3,
                                     const double *m4, const double *mo, const void *const *phi,
                                     void *const *out, double *S, const eofa_solve_params *params,
                                     eofa_solve_info *info);

/* H^{-1}(m_hi[j], m_lo[j]) phi[j] for j < n (2n chiral actions through the batch path). */
eofa_status eofa_hinv_batch(eofa_ctx *ctx, int n, const double *m_lo, const double *m_hi,
                            const void *const *phi, void *const *out, double *S,
                            const eofa_solve_params *params, eofa_solve_info *info /* 2n */);

/* Solve H_T(m_plus, m_minus) x5 = b5 (5D canonical device buffers, may not alias). */
eofa_status eofa_solve_ht(eofa_ctx *ctx, double m_plus, double m_minus, const void *b5, void *x5,
                          const eofa_solve_params *params, eofa_solve_info *info);

/*
 * eofa_apply for callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same operators, kernels and results as eofa_apply, but the
 * intermediate half fields, the site-operator tables and the reduction buffers live in a static device array
 * of 64 MiB that the library holds on every GPU it runs on until the process ends.  It calls no allocation
 * routine, and no memset or memcpy: every step is a kernel launch on the context's stream, and it returns
 * without synchronising the stream (out is ready once the stream has drained).  The context must have been
 * created and its gauge field set beforehand (those calls allocate).  The array holds eight half fields
 * (192 bytes in FP64, 96 in FP32, per 4D site of one parity and slice), four operator tables and the partial
 * sums; a lattice that does not fit is refused with EOFA_EINVAL (in FP64 up to about 43,000 site-slices per
 * parity, e.g. 8^4 with Ns = 16).  All calls on one GPU share the array and it keeps the last call's
 * contents (every call writes what it reads): calls that overlap in time on one GPU (other streams, threads
 * or contexts) race and give undefined results.
 */
eofa_status eofa_apply_static(eofa_ctx *ctx, int op, double m_plus, double m_minus, const void *in, void *out,
                              eofa_precision prec);

/*
 * Heat-bath pseudofermions (Sec. I, Eq.(CG_gaussian)): the field phi with weight exp(-S), S = phi^dag A phi for a
 * chiral action A (as in eofa_chiral_action, out = A phi), drawn from Gaussian noise eta of weight
 * exp(-eta^dag eta) as phi = A^{-1/2} P_c eta.  x^{-1/2} is replaced by Zolotarev's optimal rational
 * approximation on [lo, hi] with the fewest poles (<= 8) whose relative error is <= rel_err; each pole's term
 * (A + b)^{-1} P_c eta equals a chiral action at a shifted mass (between the action's two masses m_a < m_b) over
 * (1 + b), and all of them are solved together through the multi-RHS path under params.  lo = hi = 0 takes
 * [0.9 r, 1.1 / r], r = (1 + m_a) / (1 + m_b), which holds the spectrum on the measured fields (it is [r, 1]
 * there); a spectrum outside [lo, hi] shows in info.check.  eta, phi: 4D canonical device buffers (no alias);
 * phi's other chiral half is set to zero.
 */
typedef struct {
    int npoles;                /* poles of the rational approximation (0 when the action is the identity) */
    double approx_err;         /* its max relative error on [lo, hi] */
    double lo, hi;             /* the interval used */
    double check;              /* verify != 0: phi^dag A phi / |P_c eta|^2 - 1 (one more solve); else 0 */
    int iters_max;             /* largest iteration count of the shifted solves */
    double true_rel_resid_max; /* largest true residual of the shifted solves */
    double seconds;
} eofa_heatbath_info;
eofa_status eofa_chiral_heatbath(eofa_ctx *ctx, int chir, double m3, double m4, double mo, const void *eta,
                                 void *phi, double lo, double hi, double rel_err, int verify,
                                 const eofa_solve_params *params, eofa_heatbath_info *info);
/* phi with weight exp(-phi^dag H^{-1}(m_hi, m_lo) phi) (Eq.(Hij)): the - action (m_lo,m_lo)/(m_lo,m_hi) on the
 * P_- half of eta and the + action (m_lo,m_hi)/(m_hi,m_hi) on the P_+ half, default intervals; info[2] may be
 * NULL. */
eofa_status eofa_heatbath(eofa_ctx *ctx, double m_lo, double m_hi, const void *eta, void *phi, double rel_err,
                          int verify, const eofa_solve_params *params, eofa_heatbath_info info[2]);
/* The rational approximation above without a context (host only): x^{-1/2} ~ a0 + sum_{l < n} a[l] / (x + b[l])
 * on [lo, hi] with n <= 8 poles; *err = its max relative error on [lo, hi]. */
eofa_status eofa_inv_sqrt_rational(double lo, double hi, int n, double *a0, double *a, double *b, double *err);

/*
 * HMC molecular dynamics (Sec. I; the integrator of Sec. III).  Phase space: the links U (canonical layout,
 * periodic; the t boundary phase of the fermions is applied by the library) and the momenta
 * P[mu][site][a] (8 real components of P = P^a T^a, T^a = lambda^a / 2, site in canonical order), with
 *   H = 1/2 sum P^a P^a + S_g(U) + sum_i S_i(U),
 *   S_g = beta sum_{x, mu < nu} (1 - Re Tr U_mu nu(x) / 3)   (the Wilson plaquette action of Sec. III),
 * S_i = phi_i^dag A_i phi_i the chiral actions of an EOFA splitting (eofa_chiral_action), and the equations of
 * motion dU/dtau = i P U, dP^a/dtau = -dH/dw^a (derivative along U -> exp(i w^a T^a) U).
 */
/* S_g of the links U (device, canonical). */
eofa_status eofa_gauge_action(eofa_ctx *ctx, const void *U, double beta, double *S);
/* force[mu][site][a] = dS_g/dw^a of the links U (device, canonical); force: device, 4 * V * 8 doubles. */
eofa_status eofa_gauge_force(eofa_ctx *ctx, const void *U, double beta, double *force);

/* One pseudofermion action of the molecular dynamics: the chiral action (chir; m3, m4, mo) of
 * eofa_chiral_action on phi (4D canonical device buffer, held fixed during the trajectory), integrated on
 * time-scale level `level` (1 .. nlevels - 1; level 0 is the gauge action). */
typedef struct {
    int chir;
    double m3, m4, mo;
    int level;
    const void *phi;
} eofa_md_action;
typedef struct {
    double beta;     /* plaquette coupling */
    double tau;      /* trajectory length (Sec. III: 1) */
    int nlevels;     /* time scales, 1 .. 4 */
    int steps[4];    /* total integration steps of each level per trajectory, steps[j - 1] % (2 steps[j]) == 0;
                        Sec. III uses (k0, k1, k2) = (480, 12, 6) */
    double metropolis_u; /* in [0, 1): accept the trajectory if u < exp(-dH), else restore U; < 0: keep the end
                            point without a test */
    int chrono;          /* != 0: every force solve after an action's first in the trajectory starts from that
                            action's previous solution (kept in 2 half fields per action, allocated once) */
    double force_tol;    /* > 0: true-residual target of the force solves between the first and the last force
                            evaluation (which also give H and keep `solve`'s tol); 0: `solve`'s tol throughout */
} eofa_md_params;
typedef struct {
    double H0, H1, dH;           /* Hamiltonian at the start and the end of the trajectory */
    double K0, K1, Sg0, Sg1, Sf0, Sf1;
    int accepted;                /* 1 / 0 after a Metropolis test, -1 without one */
    int force_evals[4];          /* force evaluations per level: 2 steps[j] + 1 */
    int link_updates;
    long cg_iters;               /* CG iterations of every solve of the trajectory (forces and actions) */
    double seconds;
    /* force magnitudes, |F| = sqrt(sum_a F^a F^a) averaged over the links: per action (the first 8 of acts) the
     * largest and the mean over its force evaluations in the trajectory, and the gauge force at the start */
    double force_max[8];
    double force_mean[8];
    double gauge_force0;
} eofa_md_info;
/*
 * One molecular-dynamics trajectory from (U, P): the second-order minimum-norm (Omelyan) integrator nested over
 * time scales.  A step of level j, of size e = tau / steps[j], is
 *   P -= lam e F_j;  X_{j-1}(e/2);  P -= (1 - 2 lam) e F_j;  X_{j-1}(e/2);  P -= lam e F_j,
 * with lam = 0.1931833275037836, F_j the force of the actions of level j (F_0: the gauge force), X_{j-1}(h)
 * steps[j-1] / (2 steps[j]) steps of level j - 1 over time h, and X_{-1}(h): U <- exp(i h P) U.  Kicks of one
 * level with no link update between them see the same links and share one force evaluation (2 steps[j] + 1 per
 * level, the counts of Sec. III); the fermion actions in H at both ends come from the solves of the first and
 * last force evaluations.
 * U (device, canonical, in/out: the end point, or the start after a rejection) and P (device, in/out: the end
 * momenta) are caller-owned; every solve uses `solve`.  The context's gauge field follows U.  EINVAL for bad
 * levels, steps or arguments; a solve that does not converge stops the trajectory with its status, with U (and
 * the context's links) back at the start and P partly updated.  The library keeps one copy of the links
 * (allocated on first use).
 */
eofa_status eofa_md_trajectory(eofa_ctx *ctx, void *U, double *P, int nact, const eofa_md_action *acts,
                               const eofa_md_params *md, const eofa_solve_params *solve, eofa_md_info *info);

/* n systems H_T(m_plus[j], m_minus[j]) x5[j] = b5[j] solved together (the multi-RHS form of eofa_solve_ht; host
 * arrays of n device pointers to 5D canonical buffers, b5[j] != x5[j]).  Up to 8 systems share each launch
 * sequence, as in eofa_chiral_action_batch; info[j] per system (may be NULL). */
eofa_status eofa_solve_ht_batch(eofa_ctx *ctx, int n, const double *m_plus, const double *m_minus,
                                const void *const *b5, void *const *x5, const eofa_solve_params *params,
                                eofa_solve_info *info);

/* out = op(in) (5D canonical device buffers, may not alias) in the given storage precision
 * (EOFA_FP64 or EOFA_MIXED_FP32: FP32 storage and arithmetic, result widened to complex128). */
eofa_status eofa_apply(eofa_ctx *ctx, int op, double m_plus, double m_minus, const void *in, void *out,
                       eofa_precision prec);

/*
 * Kernel classes of one FP64 CG iteration on the even-odd normal equations (the solves that Sec. I names as
 * the cost of HMC): K1 u = A_T^{-1} H_eo p (the hop with its site-local epilogue); K2 w = Dhat p,
 * wt = A_T^{-dag} w and |w|^2; K3 at = A_T^{-dag} gamma_5 H_eo gamma_5 wt; K4 r -= alpha (w - H_oe at / 4)
 * and |r|^2; K5 x += alpha p, p = r + beta p.
 */
enum { EOFA_K_HOP = 0, EOFA_K_SCHUR_W = 1, EOFA_K_HOP_DAG = 2, EOFA_K_SCHUR_Q = 3, EOFA_K_XP = 4, EOFA_NKERN = 5 };
typedef struct {
    double ms[EOFA_NKERN];     /* summed device time, HIP events recorded on the context's stream around each launch */
    long launches[EOFA_NKERN];
    double bytes[EOFA_NKERN];  /* summed algorithmic HBM bytes: every spinor field a launch reads or writes once
                                  (12 Ns complex128 per 4D site of the output parity), its 8 links once */
} eofa_kernel_stats;
/* Per-kernel timing of the FP64 CG iterations of every later solve and eofa_cg_block: reset != 0 clears the
 * counters, enable != 0 records events from now on (a few microseconds per launch), 0 stops.  *stats (may be
 * NULL) receives the counters after the stream has drained.  Graph replays are not timed. */
eofa_status eofa_kernel_timing(eofa_ctx *ctx, int enable, int reset, eofa_kernel_stats *stats);

/*
 * Benchmark step of the FP64 solve path: the source build (R5 gamma_5 of Om (x) P_chir phi) and even-odd
 * preparation of one chiral action (chir, m3, m4 as in eofa_chiral_action; phi a 4D canonical device buffer)
 * followed by exactly niter >= 1 FP64 CG iterations on its Schur normal equations from x = 0, with no host
 * synchronisation and no convergence stop in between.  *rel (may be NULL) = |r_niter| / |r_0| of the normal
 * residual.  The solution is discarded.  Synchronises the stream.
 */
eofa_status eofa_cg_block(eofa_ctx *ctx, int chir, double m3, double m4, const void *phi, int niter, double *rel);

/* Graph replays since the context was created and the number of instantiated graphs it holds. */
eofa_status eofa_graph_stats(eofa_ctx *ctx, long *replays, int *cached);

/* Diagnostic: nrep back-to-back launches of the fused even-odd hop with its A_T^{-1} epilogue
 * (u = A_T^{-1} H_eo p, alternating parities, masses 0.01) on workspace buffers, in EOFA_FP64,
 * EOFA_MIXED_FP32 or EOFA_MIXED_FP16 storage (FP16: the batch kernel with one system, FP32 links).
 * *ms = average device time per launch (HIP events), *alg_bytes = algorithmic HBM bytes of one
 * launch (input and output half fields + 8 links per 4D site). */
eofa_status eofa_dslash_bench(eofa_ctx *ctx, int prec, int nrep, double *ms, double *alg_bytes);

/*
 * Autotuner of the hop kernels' workgroup schedule (XCD-contiguous ranges, 3D tiling of the
 * workgroup grid, and for the single-system FP64 / FP32 hop the t-walk forms, in which a workgroup
 * walks the t direction) for this lattice and storage precision (FP64, FP32 or FP16; each has its
 * own schedule, FP16 for the batch kernels): times every candidate with
 * nrep launches of the fused hop (0: 4) and keeps the fastest for all later solves.  Every
 * schedule gives bitwise the same operator; the CG reductions may sum in another order.
 * sched_out[7] (may be NULL) receives {mode, xcd, ty, tz, tt, nyb, ord} for a persistent cache
 * (mode 0: linear, 1: 3D tiles, 3: t-walk, 5: t-walk with the x neighbours from LDS, 6: mode 5 with
 * two lanes per site and slice, Ns = 16);
 * *best_ms / *base_ms (may be NULL) the chosen and the linear-order launch times.
 */
eofa_status eofa_autotune(eofa_ctx *ctx, int prec, int nrep, int sched_out[7], double *best_ms,
                          double *base_ms);
/* Re-install a schedule returned by eofa_autotune (EINVAL if it does not fit this lattice). */
eofa_status eofa_set_schedule(eofa_ctx *ctx, int prec, const int sched_in[7]);
/*
 * The schedules eofa_autotune times for this lattice and storage precision, in its order: the first
 * min(max, count) of them go to sched_out as rows of 7 ints (host memory, 7 * max ints; may be NULL
 * when max = 0), the count to *n.  No GPU work.  EINVAL for a bad prec, a null n or max < 0.
 */
eofa_status eofa_schedule_candidates(eofa_ctx *ctx, int prec, int max, int *sched_out, int *n);

/*
 * Learned preconditioner (solves with params->pc = EOFA_PC_LEARNED; Ns must be a multiple of 8).
 * A 4-layer network of 3^4 convolutions, 24 -> 32 -> 32 -> 32 -> 24 channels (spin x colour as
 * re/im), applied to the odd-site residual of the even-odd system one s-slice at a time with the
 * weights shared over s, on the checkerboard-compressed 4D lattice (xh, y, z, t) with periodic wrap.
 * It maps v to |v| N(v / |v|) and approximates (Dhat^dag Dhat)^{-1}; flexible GCR on Dhat uses
 * z = N(Dhat^dag r) as its right preconditioner.  When GCR stalls (less than 2x in |r| over 20
 * iterations) or breaks down, the solve falls back to CG on the remaining defect (info.fell_back = 1).
 * Parameters: EOFA_CNN_NPARAM FP32 values, layer by layer: weights [81 taps][32 out][32 in] (tap =
 * 27(dt+1) + 9(dz+1) + 3(dy+1) + (dx+1)), then 32 biases; entries of padded channels are ignored.
 */
#define EOFA_CNN_NPARAM (4 * (81 * 32 * 32 + 32))
/* Install parameters from host memory (count = EOFA_CNN_NPARAM); relu != 0 puts a ReLU after
 * layers 1-3 (0: linear network).  Resets the Adam state. */
eofa_status eofa_set_precond(eofa_ctx *ctx, const float *params_host, size_t count, int relu);
/* Random (He-normal, seeded) parameters; relu != 0 puts a ReLU after layers 1-3 (default: linear). */
eofa_status eofa_cnn_init(eofa_ctx *ctx, unsigned long long seed, int relu);
/* Copy the current parameters to host memory (count = EOFA_CNN_NPARAM). */
eofa_status eofa_cnn_params(eofa_ctx *ctx, float *params_host, size_t count);
/* out5 = |r| N(r / |r|) on the odd sites of the canonical 5D field in5 (even sites of out5 = 0). */
eofa_status eofa_cnn_apply(eofa_ctx *ctx, const void *in5, void *out5);
/*
 * One training pair (canonical 5D fields, odd sites used): input rho5 / |rho5|, target e5 / |rho5|,
 * loss |N - T|^2 / |T|^2 (*loss).  grad_host (may be NULL) receives dloss/dparam * |T|^2 / 2 as
 * EOFA_CNN_NPARAM floats; lr > 0 then takes one Adam step (beta = 0.9, 0.999) with that gradient.
 */
eofa_status eofa_cnn_train_step(eofa_ctx *ctx, const void *rho5, const void *e5, double lr, double *loss,
                                float *grad_host);
/*
 * Training pairs from the method's own CG: one CG solve of Dhat(m_plus, m_minus) x = b with a seeded
 * Gaussian b on the odd sites, snapshots x_k at k = 2, 4, 8, ... (n <= 16), then e_k = x* - x_k and
 * rho_k = Dhat^dag Dhat e_k, written to rho5[i] / e5[i] (canonical 5D device buffers, even sites zero).
 * *made = number of pairs written (fewer than n when CG converged early).
 */
eofa_status eofa_training_pairs(eofa_ctx *ctx, double m_plus, double m_minus, unsigned long long seed, int n,
                                void *const *rho5, void *const *e5, int *made);

const char *eofa_last_error(const eofa_ctx *ctx);
void eofa_destroy(eofa_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* EOFA_H */
