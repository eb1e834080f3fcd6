// Internal declarations shared by the kernels (kernels.hip) and the host runtime (eofa.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include "eofa_dev.h"

namespace eofa {

enum : int { HM_LIN = 0, HM_SITE = 1, HM_SCHUR_W = 2, HM_SCHUR_Q = 3, HM_DT = 4, HM_DW = 5 };

// Order in which workgroups visit the lattice (chosen per lattice by the autotuner).
// The cb index space of one parity is viewed as [t][z][yb] with yb = workgroup index along
// the (xh, y) plane line (nyb workgroups per line).  mode 0: linear.  mode 1: 3D tiles of
// ty x tz x tt workgroups visited tile by tile.  xcd != 0: every XCD (the 8 L2 domains) gets
// one contiguous range of the visiting sequence instead of every 8th workgroup.
// ord = 1 visits each tile with its (z, t) plane fastest and yb slowest.
// mode 3 (single-system FP64 / FP32 hop only): t-walk.  A workgroup owns one segment of 256 / Ns
// sites of a t-slab and walks tt consecutive slabs; the segments form an nyb x (segments / nyb) grid
// and the workgroups that run together on an XCD take a ty x tz patch of it; ord = KB of LDS reserved
// per workgroup (caps the workgroups per CU).  mode 5: mode 3 with the x-direction columns read from LDS,
// for segments that hold whole x-lines.  The other kernels read modes 3 and 5 as mode 0.
struct Sched {
    int mode, xcd, ty, tz, tt, nyb, ord;
};

template <typename R> struct HopArgs {
    Geom g;
    Sched sc;
    int par;                  // parity of the output sites
    const cpx<R>* in;         // half field of parity 1 - par (the hop input)
    const cpx<R>* Uown;       // packed links of parity par
    const cpx<R>* Uoth;       // packed links of parity 1 - par
    cpx<R>* out;
    cpx<R>* out2;
    const cpx<R>* aux;        // parity par
    const cpx<R>* aux2;       // parity par
    const cpx<R>* self;       // parity par (diagonal term of D_T / D_w)
    const SiteOp* opA;
    const SiteOp* opB;
    R cz, caux, diag;
    const double* scal;       // device scalars (alpha)
    const double* done;       // early-exit flag for graph replays (may be null)
    Red red;
};

// Multi-RHS form of the CG-iteration hops: nr independent systems (own fields, own mass tables,
// own device scalars at scal + r * SC_N) through one launch; the links of each workgroup are
// staged once and reused by all systems; a system whose SC_DONE is set is skipped.
constexpr int NRMAX = 8;
template <typename R> struct HopArgsMR {
    Geom g;
    Sched sc;
    int par, nr;
    const cpx<R>* Uown;
    const cpx<R>* Uoth;
    const cpx<R>* in[NRMAX];
    cpx<R>* out[NRMAX];
    cpx<R>* out2[NRMAX];
    const cpx<R>* aux[NRMAX];
    const cpx<R>* aux2[NRMAX];
    const SiteOp* opA[NRMAX];
    const SiteOp* opB[NRMAX];
    R cz, caux;
    double* scal;       // nr blocks of SC_N scalars
    double* partials;   // partials[r * pstride + block]
    int pstride;
    int epi;            // reduction epilogue (EPI_CG_W / EPI_CG_R) for the reducing modes
};
// half: FP16-column Krylov fields (R = float; see load_h / store_h in kernels.hip)
template <typename R> hipError_t launch_hop_mr(int Ns, bool dag, int mode, const HopArgsMR<R>& a, hipStream_t st,
                                               bool half = false);
// FP16 bytes of one half field: 12 Vh Ns (re, im) binary16 pairs + Vh Ns FP32 column norms
inline size_t half_field_bytes_h(const Geom& g, int Ns) { return (size_t)g.Vh * Ns * (12 * 4 + 4); }
// x_r (FP32) += alpha_r p_r ; p_r (FP16 columns) = r_r (FP32) + beta_r p_r, then SC_DONEX = SC_DONE
hipError_t launch_cg_xp_mr_h(int Ns, int nr, cpx<float>* const* x, void* const* p, cpx<float>* const* r, double* scal,
                             int Vh, hipStream_t st);
hipError_t launch_f2h(int Ns, const cpx<float>* in, void* out, int Vh, hipStream_t st);
hipError_t launch_h2d(int Ns, const void* in, cd* out, int Vh, hipStream_t st);
// x_r += alpha_r p_r ; p_r = r_r + beta_r p_r for the systems whose SC_DONEX is clear, then SC_DONEX = SC_DONE
template <typename R> hipError_t launch_cg_xp_mr(int nr, cpx<R>* const* x, cpx<R>* const* p, cpx<R>* const* r,
                                                 double* scal, size_t n, hipStream_t st);

template <typename R> hipError_t launch_hop(int Ns, bool dag, int mode, bool red, const HopArgs<R>& a, hipStream_t st);
int tw_grid(const Geom& g, int Ns, const Sched& sc);
template <typename R> hipError_t launch_site(int Ns, bool dag, const cpx<R>* in, cpx<R>* out, const SiteOp* op, int Vh,
                                             hipStream_t st);
// x += alpha p ; p = r + beta p unless scal[SC_DONEX] is set (follow with launch_sync_done)
template <typename R> hipError_t launch_cg_xp(cpx<R>* x, cpx<R>* p, const cpx<R>* r, double* scal, size_t n,
                                              hipStream_t st);
// for each of nr scalar blocks (stride SC_N): SC_ITERS += 1 if SC_DONEX is clear, then SC_DONEX = SC_DONE
hipError_t launch_sync_done(double* scal, int nr, hipStream_t st);
template <typename R> hipError_t launch_axpby(R a, const cpx<R>* x, R b, cpx<R>* y, size_t n, const Red* red,
                                              hipStream_t st);
template <typename R> hipError_t launch_norm2(const cpx<R>* x, size_t n, const Red& red, hipStream_t st);
// out[2i] + i out[2i+1] = <v_i, y> (complex, FP64, deterministic), i < nv <= 9; partials >= 2 nv x pstride
hipError_t launch_mdot(const cd* const* v, int nv, const cd* y, size_t n, double* partials, int pstride, double* out,
                       hipStream_t st);
// y += sum_i (cr_i + i ci_i) v_i, nv <= 9
hipError_t launch_maxpy(const cd* const* v, const double* cr, const double* ci, int nv, cd* y, size_t n, hipStream_t st);
// one-block finish of a reduction whose nblocks partials are in r.partials
hipError_t launch_finish(const Red& r, unsigned nblocks, hipStream_t st);
// dst[i] = host_vals[i], i < n <= 64 (values travel as kernel arguments: the host array may die at once)
hipError_t launch_set_vec(double* dst, int n, const double* host_vals, hipStream_t st);
// Terms of the heat-bath combination phi = a0 P_chir eta + sum_l coef[l] out[l] (canonical 4D fields).
constexpr int HB_MAXTERMS = 8;
struct HbTerms {
    const cd* out[HB_MAXTERMS];
    double coef[HB_MAXTERMS];
    double a0;
    int n;
};
// the combination over the n complex elements of a 4D field; |P_chir eta|^2 goes through red
hipError_t launch_hb_combine(const cd* eta, cd* phi, const HbTerms& t, size_t n, int chir, int accumulate,
                             const Red& red, hipStream_t st);
// dst[i] = host_vals[i] for any n, in chunks of 64 values travelling as kernel arguments
hipError_t launch_set_block(double* dst, size_t n, const double* host_vals, hipStream_t st);
// bytes (a multiple of 8) of dst set to zero / copied from src, by kernels
hipError_t launch_fill0(void* dst, size_t bytes, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// sets S[s_i] = v_i for the slots s_i >= 0 (stream-ordered, no host buffer)
hipError_t launch_scal_set(double* S, int s0, double v0, int s1, double v1, int s2, double v2, hipStream_t st);
hipError_t launch_convert_d2f(const cd* in, cpx<float>* out, size_t n, hipStream_t st);
hipError_t launch_convert_f2d(const cpx<float>* in, cd* out, size_t n, hipStream_t st);
hipError_t launch_accum_f(cd* xhi, const cpx<float>* xlo, size_t n, hipStream_t st);
template <typename R> hipError_t launch_pack5(const cd* canon, cpx<R>* half, const Geom& g, int par, int Ns, int refl,
                                              hipStream_t st);
template <typename R> hipError_t launch_unpack5(const cpx<R>* half, cd* canon, const Geom& g, int par, int Ns, int refl,
                                                hipStream_t st);
template <typename R> hipError_t launch_pack_links(const cd* U, cpx<R>* Up, const Geom& g, int par, double tbc,
                                                   hipStream_t st);
hipError_t launch_source(const cd* phi, cd* half, const Geom& g, int par, int Ns, int chir, const double* coef,
                         hipStream_t st);
hipError_t launch_combine(const cd* phi, const cd* xh, cd* out, const Geom& g, int par, int Ns, int chir, double ck,
                          const double* Om, int accumulate, const Red& red, hipStream_t st);

// ---- site-local operator tables (sitetab.cpp)
enum SiteKind : int { SK_AINV = 0, SK_AINV_DAG = 1, SK_M = 2, SK_M_DAG = 3, SK_A = 4, SK_A_DAG = 5, SK_OM1L = 6,
                      SK_OM1L_DAG = 7, SK_NKIND = 8 };
// Fill op with the tables of A_T^{-1}, A_T^{-dag}, M, M^T, A, A^T, omega (1 + L) or (1 + L)^T omega for masses
// (mp, mm).
void build_site_op(SiteOp& op, SiteKind kind, int Ns, double m0, const double* omega, double mp, double mm);

}  // namespace eofa
