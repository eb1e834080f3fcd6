// Device-side building blocks of the gfx950 EOFA / optimal-DWF path.
//
// Layout of a 5D half-lattice field (one 4D parity):  F[cb][j][s]  with
//   cb = checkerboard index of the 4D site (lexicographic index / 2),
//   j  = spin * 3 + colour (12 components), s = fifth-dimension slice (fastest).
// One work-item handles one (cb, s); the Ns work-items of a 4D site are Ns consecutive
// lanes of one 64-wide wavefront, so every s-coupling (the P+/- chain of the domain wall,
// the site-local inverse and the Om^T contraction) is a cross-lane operation inside a
// lane group: DPP row rotations when Ns = 16 (one DPP row per 4D site), ds_bpermute
// otherwise.  Reads of the 16 slices of a neighbour component are one 256-byte segment.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eofa {

// ------------------------------------------------------------------ complex helpers
template <typename R> struct alignas(2 * sizeof(R)) cpx { R x, y; };
using cd = cpx<double>;

template <typename R> __device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __device__ __forceinline__ cpx<R> cscale(R s, cpx<R> a) { return {s * a.x, s * a.y}; }
// a * b
template <typename R> __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// acc + a * b
template <typename R> __device__ __forceinline__ cpx<R> cmadd(cpx<R> acc, cpx<R> a, cpx<R> b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <typename R> __device__ __forceinline__ cpx<R> cjmadd(cpx<R> acc, cpx<R> a, cpx<R> b) {
    acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// i * a
template <typename R> __device__ __forceinline__ cpx<R> ci(cpx<R> a) { return {-a.y, a.x}; }
template <typename R> __device__ __forceinline__ cpx<R> cneg(cpx<R> a) { return {-a.x, -a.y}; }

// ------------------------------------------------------------------ lane exchange
// Value of v held by the lane (s + OFF) mod NS of this lane's group of NS lanes.
template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    int2 iv = __builtin_bit_cast(int2, v);
    iv.x = __builtin_amdgcn_mov_dpp(iv.x, CTRL, 0xF, 0xF, true);
    iv.y = __builtin_amdgcn_mov_dpp(iv.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, iv);
}

template <int NS, int OFF, typename R>
__device__ __forceinline__ R lane_from(R v, int lane) {
    if constexpr (NS == 16) {
        // row_ror:n moves lane (i - n) mod 16 into lane i; we want source i + OFF.
        constexpr int n = ((16 - OFF) % 16 + 16) % 16;
        static_assert(n != 0, "zero rotation");
        if constexpr (sizeof(R) == 8) return dpp_d<0x120 + n>(v);
        else return dpp_f<0x120 + n>(v);
    } else {
        int src = (lane & ~(NS - 1)) | ((lane + OFF) & (NS - 1));
        return __shfl(v, src, 64);
    }
}

template <int NS, int OFF, typename R>
__device__ __forceinline__ cpx<R> lane_from_c(cpx<R> v, int lane) {
    return {lane_from<NS, OFF>(v.x, lane), lane_from<NS, OFF>(v.y, lane)};
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// ------------------------------------------------------------------ site-local s-operators
// Tables of one chirality half of a site-local operator (see sitetab.cpp for the algebra).
// Every op has the shape  post * [ shift and/or cyclic bidiagonal solve ] * pre  with
//   solve: x_s = g_s + c_s x_{s+sig} around the ring, done as a log2(Ns)-step ring scan
//          B_s += q[k][s] * B_{s + 2^k sig}, and x = kappa * B (kappa folded into post);
//   shift: y_s = x_s + shf[s] * x_{s+sig}.
constexpr int MAXNS = 64;
struct ChirTab {
    double pre[MAXNS];
    double mid[MAXNS];
    double q[6][MAXNS];
    double shf[MAXNS];
    double post[MAXNS];
};
// One site-local operator = tables for the upper (P+) and lower (P-) spin halves.
struct SiteOp { ChirTab h[2]; };

// A copy of the first NS entries of a ChirTab / SiteOp, staged by a workgroup in LDS (stage_siteop).
template <int NS> struct ChirTabL {
    double pre[NS];
    double mid[NS];
    double shf[NS];
    double post[NS];
    double q[ilog2(NS) > 0 ? ilog2(NS) : 1][NS];
};
template <int NS> struct SiteOpL { ChirTabL<NS> h[2]; };

// Staging of a SiteOp into LDS by a workgroup of 256 lanes, in two halves so that the caller can issue
// other loads between them: siteop_fetch loads this lane's share into registers, siteop_store writes it
// to d (published by the caller's next workgroup barrier).
template <int NS> struct SiteOpShare {
    static constexpr int L = ilog2(NS) > 0 ? ilog2(NS) : 1;
    static constexpr int F = 4 + L, TOT = 2 * F * NS, NQ = (TOT + 255) / 256;
    double v[NQ];
};

template <int NS>
__device__ __forceinline__ void siteop_fetch(SiteOpShare<NS>& sh, const SiteOp& op) {
    using S = SiteOpShare<NS>;
#pragma unroll
    for (int k = 0; k < S::NQ; k++) {
        const int e = min((int)threadIdx.x + 256 * k, S::TOT - 1);  // lanes past the end repeat the last entry
        const int hf = e / (S::F * NS), f = (e / NS) % S::F, si = e % NS;
        const double* row = f == 0 ? op.h[hf].pre : f == 1 ? op.h[hf].mid : f == 2 ? op.h[hf].shf
                          : f == 3 ? op.h[hf].post : op.h[hf].q[f - 4];
        sh.v[k] = row[si];
    }
}

template <int NS>
__device__ __forceinline__ void siteop_store(SiteOpL<NS>& d, const SiteOpShare<NS>& sh) {
    using S = SiteOpShare<NS>;
    static_assert(sizeof(ChirTabL<NS>) == sizeof(double) * S::F * NS, "ChirTabL layout");
    double* flat = &d.h[0].pre[0];  // h[hf] rows pre, mid, shf, post, q[0..L) are contiguous
#pragma unroll
    for (int k = 0; k < S::NQ; k++) {
        const int e = threadIdx.x + 256 * k;
        if (e < S::TOT) flat[e] = sh.v[k];
    }
}

// NC: the number of colour-spin components of the chirality half held by this lane (6, or 3 when the two
// spins of a half sit in two lanes); every component is transformed independently.
template <int NS, int SIG, int K, int NC = 6, typename R, typename T>
__device__ __forceinline__ void ring_scan_step(cpx<R> v[NC], const T& t, int s, int lane) {
    if constexpr (K < ilog2(NS)) {
        const R qk = (R)t.q[K][s];
        constexpr int OFF = SIG * (1 << K);
#pragma unroll
        for (int j = 0; j < NC; j++) {
            cpx<R> o = lane_from_c<NS, OFF>(v[j], lane);
            v[j].x = fma(qk, o.x, v[j].x);
            v[j].y = fma(qk, o.y, v[j].y);
        }
        ring_scan_step<NS, SIG, K + 1, NC>(v, t, s, lane);
    }
}

// ORDER 0: solve then shift (A^{-1}-type ops).  ORDER 1: shift then solve (their transposes).
template <int NS, int SIG, int ORDER, int NC = 6, typename R, typename T>
__device__ __forceinline__ void chir_op(cpx<R> v[NC], const T& t, int s, int lane) {
    const R pre = (R)t.pre[s], post = (R)t.post[s], shf = (R)t.shf[s];
#pragma unroll
    for (int j = 0; j < NC; j++) v[j] = cscale(pre, v[j]);
    if constexpr (ORDER == 0) {
        ring_scan_step<NS, SIG, 0, NC>(v, t, s, lane);
#pragma unroll
        for (int j = 0; j < NC; j++) {
            cpx<R> o = lane_from_c<NS, SIG>(v[j], lane);
            v[j].x = post * fma(shf, o.x, v[j].x);
            v[j].y = post * fma(shf, o.y, v[j].y);
        }
    } else {
        const R mid = (R)t.mid[s];
#pragma unroll
        for (int j = 0; j < NC; j++) {
            cpx<R> o = lane_from_c<NS, SIG>(v[j], lane);
            v[j].x = mid * fma(shf, o.x, v[j].x);
            v[j].y = mid * fma(shf, o.y, v[j].y);
        }
        ring_scan_step<NS, SIG, 0, NC>(v, t, s, lane);
#pragma unroll
        for (int j = 0; j < NC; j++) v[j] = cscale(post, v[j]);
    }
}

// Apply a site-local operator to a 12-component spinor held lane-wise over s.
// DAG = false: upper half couples s to s-1 (L_+), lower to s+1 (L_-); DAG = true reverses both.
template <int NS, bool DAG, typename R, typename Op>
__device__ __forceinline__ void site_op(cpx<R> v[12], const Op& op, int s, int lane) {
    constexpr int SU = DAG ? +1 : -1;
    constexpr int ORD = DAG ? 1 : 0;
    chir_op<NS, SU, ORD>(v, op.h[0], s, lane);
    chir_op<NS, -SU, ORD>(v + 6, op.h[1], s, lane);
}

// The same operator on one upper spin v[0..2] and one lower spin v[3..5] (3 colours each): the share of a lane
// of the spin-split hop, whose partner lane holds the other spin of each half.
template <int NS, bool DAG, typename R, typename Op>
__device__ __forceinline__ void site_op_half(cpx<R> v[6], const Op& op, int s, int lane) {
    constexpr int SU = DAG ? +1 : -1;
    constexpr int ORD = DAG ? 1 : 0;
    chir_op<NS, SU, ORD, 3>(v, op.h[0], s, lane);
    chir_op<NS, -SU, ORD, 3>(v + 3, op.h[1], s, lane);
}

// ------------------------------------------------------------------ spin projection (chiral basis)
// gamma_mu = [[0, B_mu], [B_mu^dag, 0]] with B_k = -i sigma_k (k = x, y, z) and B_t = 1.
// (1 + S gamma_mu) psi = [h ; S B^dag h] with h = psi_up + S B psi_dn, so only the 2-spinor h
// is multiplied by the link.
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cpx<R> p[12], cpx<R> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cpx<R> d0 = p[6 + c], d1 = p[9 + c], b0, b1;
        if constexpr (MU == 0) { b0 = cneg(ci(d1)); b1 = cneg(ci(d0)); }
        else if constexpr (MU == 1) { b0 = cneg(d1); b1 = d0; }
        else if constexpr (MU == 2) { b0 = cneg(ci(d0)); b1 = ci(d1); }
        else { b0 = d0; b1 = d1; }
        if constexpr (S > 0) { h[c] = cadd(p[c], b0); h[3 + c] = cadd(p[3 + c], b1); }
        else { h[c] = csub(p[c], b0); h[3 + c] = csub(p[3 + c], b1); }
    }
}

template <int MU, int S, typename R>
__device__ __forceinline__ void reconstruct(cpx<R> acc[12], const cpx<R> w[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cpx<R> w0 = w[c], w1 = w[3 + c], t0, t1;  // t = B^dag w
        if constexpr (MU == 0) { t0 = ci(w1); t1 = ci(w0); }
        else if constexpr (MU == 1) { t0 = w1; t1 = cneg(w0); }
        else if constexpr (MU == 2) { t0 = ci(w0); t1 = cneg(ci(w1)); }
        else { t0 = w0; t1 = w1; }
        acc[c] = cadd(acc[c], w0);
        acc[3 + c] = cadd(acc[3 + c], w1);
        if constexpr (S > 0) { acc[6 + c] = cadd(acc[6 + c], t0); acc[9 + c] = cadd(acc[9 + c], t1); }
        else { acc[6 + c] = csub(acc[6 + c], t0); acc[9 + c] = csub(acc[9 + c], t1); }
    }
}

// w = U h (ADJ = false) or U^dag h (ADJ = true) for the two spin components of h.
template <bool ADJ, typename R>
__device__ __forceinline__ void link_mul(const cpx<R> U[9], const cpx<R> h[6], cpx<R> w[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int r = 0; r < 3; r++) {
            cpx<R> a = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) {
                if constexpr (!ADJ) a = cmadd(a, U[3 * r + k], h[3 * sp + k]);
                else a = cjmadd(a, U[3 * k + r], h[3 * sp + k]);
            }
            w[3 * sp + r] = a;
        }
}

// ------------------------------------------------------------------ lattice geometry
struct Geom {
    int Lx, Ly, Lz, Lt;  // full extents
    int Lxh;             // Lx / 2
    int Vh;              // 4D sites per parity
};

// Neighbour checkerboard indices of the 4D site cb of parity par.  nb[2*mu] = x+mu, nb[2*mu+1] = x-mu.
__device__ __forceinline__ void neighbours(const Geom& g, int cb, int par, int nb[8]) {
    int xh = cb % g.Lxh;
    int r = cb / g.Lxh;
    int y = r % g.Ly; r /= g.Ly;
    int z = r % g.Lz;
    int t = r / g.Lz;
    int x = 2 * xh + ((y + z + t + par) & 1);
    int base = cb - xh;  // cb of (x = 0|1, y, z, t)
    int xp = (x + 1 == g.Lx) ? 0 : x + 1;
    int xm = (x == 0) ? g.Lx - 1 : x - 1;
    nb[0] = base + (xp >> 1);
    nb[1] = base + (xm >> 1);
    int sy = g.Lxh, sz = g.Lxh * g.Ly, st = sz * g.Lz;
    nb[2] = (y + 1 == g.Ly) ? cb - (g.Ly - 1) * sy : cb + sy;
    nb[3] = (y == 0) ? cb + (g.Ly - 1) * sy : cb - sy;
    nb[4] = (z + 1 == g.Lz) ? cb - (g.Lz - 1) * sz : cb + sz;
    nb[5] = (z == 0) ? cb + (g.Lz - 1) * sz : cb - sz;
    nb[6] = (t + 1 == g.Lt) ? cb - (g.Lt - 1) * st : cb + st;
    nb[7] = (t == 0) ? cb + (g.Lt - 1) * st : cb - st;
}

// ------------------------------------------------------------------ deterministic reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum (blockDim.x == 256); result valid in every thread.
__device__ __forceinline__ double block_sum256(double v, double* lds4) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds4[w] = v;
    __syncthreads();
    return (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
}

// Reduction: every block writes its partial sum; a one-block finishing kernel (k_finish)
// adds the partials in a fixed order and applies an epilogue to the device scalars.  No
// atomics and no cross-XCD fences inside the producing kernel; the result is bitwise
// reproducible run to run.
struct Red {
    double* partials;   // >= gridDim.x doubles
    double* scal;       // device scalars
    int slot;           // where the sum goes
    int epi;            // epilogue (see finish_partials)
};

enum : int {
    SC_RR = 0,      // |r|^2 of the running CG
    SC_WW = 1,      // |Dhat p|^2
    SC_ALPHA = 2,
    SC_BETA = 3,
    SC_RR0 = 4,     // |r_0|^2 (stop reference)
    SC_DONE = 5,    // 1 when converged (read by graph replays)
    SC_TOL2 = 6,    // stop threshold on |r|^2 / |r_0|^2
    SC_DONEX = 7,   // the x/p update of the converged iteration has been applied (lags SC_DONE by one kernel)
    SC_TMP = 8,     // 8..29 free slots for norms
    SC_ITERS = 30,  // CG iterations applied since the counter was cleared (counted on the device)
    SC_N = 32
};
enum : int { EPI_STORE = 0, EPI_CG_W = 1, EPI_CG_R = 2, EPI_CG_INIT = 3 };

// Called by every thread of every block with the block's sum (same value in all threads).
__device__ __forceinline__ void finish_sum(const Red& rd, double bsum) {
    if (threadIdx.x == 0) rd.partials[blockIdx.x] = bsum;
}

// Sum partials[0..n) in a fixed order (256 threads) and apply the epilogue.
__device__ __forceinline__ void finish_partials(const double* partials, unsigned n, double* S, int slot, int epi) {
    __shared__ double lds[4];
    // 8 independent loads in flight per thread; the summation order is fixed
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned i = threadIdx.x;
    for (; i + 7 * 256 < n; i += 8 * 256)
#pragma unroll
        for (int k = 0; k < 8; k++) a[k] += partials[i + k * 256];
    for (; i < n; i += 256) a[0] += partials[i];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    s = block_sum256(s, lds);
    if (threadIdx.x == 0) {
        switch (epi) {
        case EPI_CG_W:          // s = |Dhat p|^2 (after convergence the hops were skipped: keep the scalars)
            if (S[SC_DONE] != 0.0) break;
            S[SC_WW] = s;
            S[SC_ALPHA] = S[SC_RR] / s;
            break;
        case EPI_CG_R:          // s = |r_new|^2
            if (S[SC_DONE] != 0.0) break;
            S[SC_BETA] = s / S[SC_RR];
            S[SC_RR] = s;
            if (s <= S[SC_TOL2] * S[SC_RR0]) S[SC_DONE] = 1.0;
            break;
        case EPI_CG_INIT:       // s = |r_0|^2
            S[SC_RR] = s;
            S[SC_RR0] = s;
            S[SC_DONE] = (s == 0.0) ? 1.0 : 0.0;
            S[SC_DONEX] = S[SC_DONE];
            S[SC_ITERS] = 0.0;
            break;
        default:
            S[slot] = s;
        }
    }
}

}  // namespace eofa
