// gfx950 kernels of the EOFA / optimal-DWF solve path: the fused even-odd hop with its
// site-local epilogues, BLAS-1 steps with deterministic FP64 reductions, and the
// pack / source / combine kernels at the canonical boundary.
#include <algorithm>

#include "eofa_int.h"

namespace eofa {

// ===================================================================== the fused hop
// One launch computes, for every (4D site x of parity par, slice s):
//   z = sum_mu [(1 - S gamma_mu) U_mu(x) in(x+mu, s) + (1 + S gamma_mu) U_mu(x-mu)^dag in(x-mu, s)]
// (S = +1 normal hop, S = -1 for gamma_5 hop gamma_5 when DAG) and then one epilogue:
//   HM_LIN     out = caux*aux + cz*z
//   HM_SITE    out = A (caux*aux + cz*z)                       A = site op (A_T^{-1} or A_T^{-dag})
//   HM_SCHUR_W out = w = caux*aux + cz*A(z);  out2 = B(w);  sum |w|^2 -> alpha   (Dhat p, A^{-dag} Dhat p)
//   HM_SCHUR_Q q = caux*aux + cz*z;  out = aux2 - alpha*q;  sum |out|^2 -> beta  (CG residual update)
//   HM_DT      out = caux*aux + cz*((4-m0) self + A(self) - z/2)                (D_T, A = M or M^T)
//   HM_DW      out = caux*aux + cz*((4-m0) self - z/2)                          (D_w on every slice)
// Scheduling fence between the directions of the hop: keeps the compiler from hoisting every neighbour load
// to the top (which spills at 256 VGPRs in FP64).
#define HOP_FENCE() __builtin_amdgcn_sched_barrier(0)

// Cache policy of the hop's outputs: they are not read again by the same launch, so they bypass the
// caches that hold the re-read neighbour spinors.
template <typename R> __device__ __forceinline__ void st_out(cpx<R>* p, const cpx<R>& v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}
template <typename T> __device__ __forceinline__ void st_raw(T* p, const T& v) { __builtin_nontemporal_store(v, p); }
// The epilogues' site-local inputs (aux, aux2) are read once per launch: nontemporal loads, so that they do not
// displace the re-read neighbour spinors either.
template <typename R> __device__ __forceinline__ cpx<R> ld_once(const cpx<R>* p) {
    return {__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}

// ---- FP16 storage of a Krylov half field (EOFA_MIXED_FP16): per (cb, s) column the 12 complex
// components as binary16 (re, im) pairs in 3 blocks of 4 (16 bytes, one load per block):
// F[cb][jb < 3][Ns][4 pairs], each column scaled by its own FP32 norm = the largest |real component| of
// its 24 reals, stored after the 12 Vh Ns pairs.  value = norm * half, |half| <= 1.
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));

template <int NS> __device__ __forceinline__ const float* h_norms(const void* f, int Vh) {
    return (const float*)((const h8_t*)f + (size_t)3 * Vh * NS);
}

// NT: nontemporal loads (a column read once per launch)
template <int NS, bool NT = false>
__device__ __forceinline__ void load_h(cpx<float> p[12], const void* __restrict__ f, size_t cb, int s, int Vh) {
    const h8_t* d = (const h8_t*)f + cb * 3 * NS + s;
    const float* np = h_norms<NS>(f, Vh) + cb * NS + s;
    const float n = NT ? __builtin_nontemporal_load(np) : *np;
#pragma unroll
    for (int jb = 0; jb < 3; jb++) {
        const h8_t v = NT ? __builtin_nontemporal_load(d + jb * NS) : d[jb * NS];
#pragma unroll
        for (int k = 0; k < 4; k++) p[4 * jb + k] = {n * (float)v[2 * k], n * (float)v[2 * k + 1]};
    }
}

template <int NS>
__device__ __forceinline__ void store_h(void* __restrict__ f, size_t cb, int s, int Vh, const cpx<float> v[12]) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < 12; j++) m = fmaxf(m, fmaxf(fabsf(v[j].x), fabsf(v[j].y)));
    const float inv = m > 0.0f ? 1.0f / m : 0.0f;
    h8_t* d = (h8_t*)f + cb * 3 * NS + s;
#pragma unroll
    for (int jb = 0; jb < 3; jb++) {
        h8_t h;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            h[2 * k] = (_Float16)(v[4 * jb + k].x * inv);
            h[2 * k + 1] = (_Float16)(v[4 * jb + k].y * inv);
        }
        st_raw(d + jb * NS, h);
    }
    st_raw((float*)h_norms<NS>(f, Vh) + cb * NS + s, m);
}

// 12 components of (cb, s) from a field in storage H (FP16 columns) or plain cpx<R>; NT: nontemporal loads
template <int NS, bool H, bool NT = false, typename R>
__device__ __forceinline__ void load_col(cpx<R> p[12], const void* __restrict__ f, size_t cb, int s, int Vh) {
    if constexpr (H) {
        load_h<NS, NT>(p, f, cb, s, Vh);
    } else {
        const cpx<R>* src = (const cpx<R>*)f + cb * 12 * NS + s;
#pragma unroll
        for (int j = 0; j < 12; j++) p[j] = NT ? ld_once(src + j * NS) : src[j * NS];
    }
}

template <int NS, bool H, typename R>
__device__ __forceinline__ void store_col(void* __restrict__ f, size_t cb, int s, int Vh, const cpx<R> v[12]) {
    if constexpr (H) {
        store_h<NS>(f, cb, s, Vh, v);
    } else {
        cpx<R>* dst = (cpx<R>*)f + cb * 12 * NS + s;
#pragma unroll
        for (int j = 0; j < 12; j++) st_out(dst + j * NS, v[j]);
    }
}

// An FP16 column of a field in storage H without its norm (p = raw binary16 values widened) and the norm n.
template <int NS>
__device__ __forceinline__ float load_h_raw(cpx<float> p[12], const void* __restrict__ f, size_t cb, int s, int Vh) {
    const h8_t* d = (const h8_t*)f + cb * 3 * NS + s;
#pragma unroll
    for (int jb = 0; jb < 3; jb++) {
        const h8_t v = d[jb * NS];
#pragma unroll
        for (int k = 0; k < 4; k++) p[4 * jb + k] = {(float)v[2 * k], (float)v[2 * k + 1]};
    }
    return h_norms<NS>(f, Vh)[cb * NS + s];
}

// reconstruct() of n w: the column norm of an FP16 neighbour folded into the accumulation (one FMA per real
// instead of a multiply on every loaded component and an add)
template <int MU, int S, typename R>
__device__ __forceinline__ void reconstruct_n(cpx<R> acc[12], const cpx<R> w[6], R n) {
    const R sn = S > 0 ? n : -n;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cpx<R> w0 = w[c], w1 = w[3 + c], t0, t1;  // t = B^dag w
        if constexpr (MU == 0) { t0 = ci(w1); t1 = ci(w0); }
        else if constexpr (MU == 1) { t0 = w1; t1 = cneg(w0); }
        else if constexpr (MU == 2) { t0 = ci(w0); t1 = cneg(ci(w1)); }
        else { t0 = w0; t1 = w1; }
        acc[c].x = fma(n, w0.x, acc[c].x); acc[c].y = fma(n, w0.y, acc[c].y);
        acc[3 + c].x = fma(n, w1.x, acc[3 + c].x); acc[3 + c].y = fma(n, w1.y, acc[3 + c].y);
        acc[6 + c].x = fma(sn, t0.x, acc[6 + c].x); acc[6 + c].y = fma(sn, t0.y, acc[6 + c].y);
        acc[9 + c].x = fma(sn, t1.x, acc[9 + c].x); acc[9 + c].y = fma(sn, t1.y, acc[9 + c].y);
    }
}

// One direction mu of the hop: forward (1 - S gamma) U in(x+mu) and backward (1 + S gamma) U^dag in(x-mu).
// Uf / Ub point at the 9 complex entries of U_mu(x) and U_mu(x-mu) (global memory or LDS).  FP16 columns (H)
// are projected and multiplied unscaled; their norm enters in the accumulation.
template <int NS, bool DAG, int MU, typename R, bool H = false>
__device__ __forceinline__ void hop_mu(cpx<R> acc[12], const cpx<R>* __restrict__ in, const cpx<R>* Uf,
                                       const cpx<R>* Ub, const int nb[8], int s, int Vh = 0) {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    {
        cpx<R> p[12];
        R n = 1;
        if constexpr (H) n = load_h_raw<NS>(p, in, (size_t)nb[2 * MU], s, Vh);
        else load_col<NS, H>(p, in, (size_t)nb[2 * MU], s, Vh);
        cpx<R> h[6], w[6], U[9];
        project<MU, SF>(p, h);
#pragma unroll
        for (int k = 0; k < 9; k++) U[k] = Uf[k];
        link_mul<false>(U, h, w);
        if constexpr (H) reconstruct_n<MU, SF>(acc, w, n);
        else reconstruct<MU, SF>(acc, w);
    }
    {
        cpx<R> p[12];
        R n = 1;
        if constexpr (H) n = load_h_raw<NS>(p, in, (size_t)nb[2 * MU + 1], s, Vh);
        else load_col<NS, H>(p, in, (size_t)nb[2 * MU + 1], s, Vh);
        cpx<R> h[6], w[6], U[9];
        project<MU, SB>(p, h);
#pragma unroll
        for (int k = 0; k < 9; k++) U[k] = Ub[k];
        link_mul<true>(U, h, w);
        if constexpr (H) reconstruct_n<MU, SB>(acc, w, n);
        else reconstruct<MU, SB>(acc, w);
    }
}

// The 8 links of each of the workgroup's 256/NS sites, staged in LDS: sU[site][l][k], l = 0..3 the
// forward links U_mu(x), l = 4..7 the backward links U_mu(x - mu).  Each entry is read once from
// global memory instead of once per slice.  Ends with a workgroup barrier.
struct NoStore {
    __device__ void operator()() const {}
};
// between issuing its loads and writing LDS it runs more_stores (LDS writes of other staged data whose
// loads were issued before, so that one memory round trip covers both).
// TW: slot 7 holds U_t of the input site x + t instead of U_t(x - t) (the t-walk's carry link).
template <int NS, typename R, typename F = NoStore, bool TW = false>
__device__ __forceinline__ void stage_links(cpx<R> (*sU)[8][9], const cpx<R>* __restrict__ Uown,
                                            const cpx<R>* __restrict__ Uoth, int cb, const int nb[8], int s,
                                            F more_stores = F()) {
    const int ls = threadIdx.x / NS;
    constexpr int NQ = (72 + NS - 1) / NS;
    // complex entries moved as 2-vectors: whole-struct copies through a private array are lowered to
    // memcpy, which can keep the array in scratch memory
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {  // every load in flight before the first LDS write; no branches
        const int e = min(s + q * NS, 71), l = e / 9, k = e % 9;
        // selects, not nb[2 * (l - 4) + 1]: a runtime index would move nb out of registers
        const int nbl = l == 4 ? nb[1] : l == 5 ? nb[3] : l == 6 ? nb[5] : (TW ? nb[6] : nb[7]);
        const cpx<R>* src = (l < 4) ? Uown + ((size_t)cb * 4 + l) * 9 + k : Uoth + ((size_t)nbl * 4 + (l - 4)) * 9 + k;
        v[q] = *(const v2*)src;
    }
    more_stores();
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int e = s + q * NS;
        if (e < 72) *(v2*)&sU[ls][e / 9][e % 9] = v[q];
    }
    __syncthreads();
}

// z = hop(in) at (cb, s) with the links of this lane's site in sUl[8][9].
template <int NS, bool DAG, typename R, bool H = false>
__device__ __forceinline__ void hop_lds(cpx<R> z[12], const cpx<R>* __restrict__ in, const cpx<R> (*sUl)[9],
                                        const int nb[8], int s, int Vh = 0) {
#pragma unroll
    for (int j = 0; j < 12; j++) z[j] = {0, 0};
    hop_mu<NS, DAG, 0, R, H>(z, in, sUl[0], sUl[4], nb, s, Vh);
    HOP_FENCE();
    hop_mu<NS, DAG, 1, R, H>(z, in, sUl[1], sUl[5], nb, s, Vh);
    HOP_FENCE();
    hop_mu<NS, DAG, 2, R, H>(z, in, sUl[2], sUl[6], nb, s, Vh);
    HOP_FENCE();
    hop_mu<NS, DAG, 3, R, H>(z, in, sUl[3], sUl[7], nb, s, Vh);
}

// z = hop(in) at (cb, s).  For Ns >= 8 the workgroup first stages its sites' links in LDS (each link is then
// read once instead of once per slice); Ns = 4 reads them from global memory.  more_stores runs once before
// the workgroup barrier that publishes the staged data.
template <int NS, bool DAG, typename R, typename F>
__device__ __forceinline__ void hop_all(cpx<R> z[12], const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ Uown,
                                        const cpx<R>* __restrict__ Uoth, int cb, const int nb[8], int s,
                                        F more_stores) {
    if constexpr (NS >= 8) {
        __shared__ cpx<R> sU[256 / NS][8][9];
        stage_links<NS>(sU, Uown, Uoth, cb, nb, s, more_stores);
        hop_lds<NS, DAG>(z, in, sU[threadIdx.x / NS], nb, s);
    } else {
        more_stores();
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 12; j++) z[j] = {0, 0};
        hop_mu<NS, DAG, 0>(z, in, Uown + ((size_t)cb * 4 + 0) * 9, Uoth + ((size_t)nb[1] * 4 + 0) * 9, nb, s);
        HOP_FENCE();
        hop_mu<NS, DAG, 1>(z, in, Uown + ((size_t)cb * 4 + 1) * 9, Uoth + ((size_t)nb[3] * 4 + 1) * 9, nb, s);
        HOP_FENCE();
        hop_mu<NS, DAG, 2>(z, in, Uown + ((size_t)cb * 4 + 2) * 9, Uoth + ((size_t)nb[5] * 4 + 2) * 9, nb, s);
        HOP_FENCE();
        hop_mu<NS, DAG, 3>(z, in, Uown + ((size_t)cb * 4 + 3) * 9, Uoth + ((size_t)nb[7] * 4 + 3) * 9, nb, s);
    }
}

// v += c * aux[j * NS] for the 12 components (aux already offset to this lane's element)
template <int NS, typename R>
__device__ __forceinline__ void add_aux_ns(cpx<R> v[12], const cpx<R>* __restrict__ aux, R c) {
#pragma unroll
    for (int j = 0; j < 12; j++) {
        cpx<R> t = ld_once(aux + j * NS);
        v[j].x = fma(c, t.x, v[j].x);
        v[j].y = fma(c, t.y, v[j].y);
    }
}
#define add_aux(v, ptr, c) add_aux_ns<NS>(v, ptr, c)

// Workgroup -> tile of 256 lanes, following the schedule (see Sched).
__device__ __forceinline__ int tile_of(int b, int n, const Sched& sc, const Geom& g) {
    if (sc.xcd) {  // hardware dispatches workgroup b to XCD b % 8
        const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
        b = x * q + (x < r ? x : r) + i;
    }
    if (sc.mode == 1) {
        const int per = sc.ty * sc.tz * sc.tt;
        const int intra = b % per, tile = b / per;
        const int nyt = sc.nyb / sc.ty, nzt = g.Lz / sc.tz;
        int yy, zz, tq;
        if (sc.ord) { zz = intra % sc.tz; tq = (intra / sc.tz) % sc.tt; yy = intra / (sc.tz * sc.tt); }
        else { yy = intra % sc.ty; zz = (intra / sc.ty) % sc.tz; tq = intra / (sc.ty * sc.tz); }
        const int ty = tile % nyt, tz = (tile / nyt) % nzt, tt = tile / (nyt * nzt);
        const int yb = ty * sc.ty + yy, z = tz * sc.tz + zz, t = tt * sc.tt + tq;
        b = yb + sc.nyb * (z + g.Lz * t);
    }
    return b;
}
// occupancy hint of the hop kernels: 2 workgroups of 256 lanes per CU (128 VGPRs would spill in FP64)
constexpr int HOP_WAVES = 2;

// The epilogue of the fused hop at (cb, s) given z = hop(in): stores out (and out2 for HM_SCHUR_W) when
// valid and returns this lane's contribution to the reduced norm (0 unless RED).  opA / opB are the
// site-local operators (LDS copies).
template <int NS, bool DAG, int MODE, bool RED, typename R, typename TA, typename TB>
__device__ __forceinline__ double hop_epilogue(const HopArgs<R>& a, cpx<R> z[12], int cb, int s, int lane,
                                               bool valid, const TA& opA, const TB& opB) {
    const size_t base = (size_t)cb * 12 * NS + s;
    double nrm = 0.0;
    cpx<R> v[12];
    if constexpr (MODE == HM_LIN || MODE == HM_SITE) {
#pragma unroll
        for (int j = 0; j < 12; j++) v[j] = cscale(a.cz, z[j]);
        if (a.aux) add_aux(v, a.aux + base, a.caux);
        if constexpr (MODE == HM_SITE) site_op<NS, DAG>(v, opA, s, lane);
    } else if constexpr (MODE == HM_SCHUR_W) {
        site_op<NS, false>(z, opA, s, lane);
#pragma unroll
        for (int j = 0; j < 12; j++) {
            cpx<R> t = ld_once(a.aux + base + j * NS);
            v[j].x = fma(a.cz, z[j].x, a.caux * t.x);
            v[j].y = fma(a.cz, z[j].y, a.caux * t.y);
        }
    } else if constexpr (MODE == HM_SCHUR_Q) {
        const R alpha = (R)a.scal[SC_ALPHA];
#pragma unroll
        for (int j = 0; j < 12; j++) {
            cpx<R> w = ld_once(a.aux + base + j * NS), r = ld_once(a.aux2 + base + j * NS);
            R qx = fma(a.cz, z[j].x, a.caux * w.x), qy = fma(a.cz, z[j].y, a.caux * w.y);
            v[j].x = fma(-alpha, qx, r.x);
            v[j].y = fma(-alpha, qy, r.y);
        }
    } else if constexpr (MODE == HM_DT || MODE == HM_DW) {
        cpx<R> d[12];
#pragma unroll
        for (int j = 0; j < 12; j++) d[j] = a.self[base + j * NS];
        cpx<R> m[12];
#pragma unroll
        for (int j = 0; j < 12; j++) m[j] = d[j];
        if constexpr (MODE == HM_DT) site_op<NS, DAG>(m, opA, s, lane);
#pragma unroll
        for (int j = 0; j < 12; j++) {
            R tx = a.diag * d[j].x - (R)0.5 * z[j].x, ty = a.diag * d[j].y - (R)0.5 * z[j].y;
            if constexpr (MODE == HM_DT) { tx += m[j].x; ty += m[j].y; }
            v[j] = {a.cz * tx, a.cz * ty};
        }
        if (a.aux) add_aux(v, a.aux + base, a.caux);
    }
    if (valid) {
#pragma unroll
        for (int j = 0; j < 12; j++) st_out(a.out + base + j * NS, v[j]);
    }
    if constexpr (MODE == HM_SCHUR_W) {
        if constexpr (RED) {
#pragma unroll
            for (int j = 0; j < 12; j++) nrm += (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
        }
        site_op<NS, true>(v, opB, s, lane);
        if (valid) {
#pragma unroll
            for (int j = 0; j < 12; j++) st_out(a.out2 + base + j * NS, v[j]);
        }
    } else if constexpr (RED) {
#pragma unroll
        for (int j = 0; j < 12; j++) nrm += (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
    }
    return valid ? nrm : 0.0;
}

// LDS copies of the site-local operators the epilogue of MODE applies: ops_fetch issues the loads,
// ops_store writes the copies (published by the next barrier).
template <int NS> struct OpsShare { SiteOpShare<NS> A, B; };
template <int NS, int MODE, typename R>
__device__ __forceinline__ void ops_fetch(OpsShare<NS>& sh, const HopArgs<R>& a) {
    if constexpr (MODE == HM_SITE || MODE == HM_SCHUR_W || MODE == HM_DT) siteop_fetch<NS>(sh.A, *a.opA);
    if constexpr (MODE == HM_SCHUR_W) siteop_fetch<NS>(sh.B, *a.opB);
}
template <int NS, int MODE>
__device__ __forceinline__ void ops_store(SiteOpL<NS>& sA, SiteOpL<NS>& sB, const OpsShare<NS>& sh) {
    if constexpr (MODE == HM_SITE || MODE == HM_SCHUR_W || MODE == HM_DT) siteop_store<NS>(sA, sh.A);
    if constexpr (MODE == HM_SCHUR_W) siteop_store<NS>(sB, sh.B);
}

template <int NS, bool DAG, int MODE, bool RED, typename R>
__global__ __launch_bounds__(256, HOP_WAVES) void k_hop(const HopArgs<R> a) {
    if (a.done && *a.done != 0.0) return;
    const int tid = tile_of(blockIdx.x, gridDim.x, a.sc, a.g) * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int s = lane & (NS - 1);
    int cb = tid / NS;
    const bool valid = cb < a.g.Vh;
    if (!valid) cb = a.g.Vh - 1;  // keep every lane of a group active for the lane exchanges
    int nb[8];
    neighbours(a.g, cb, a.par, nb);
    __shared__ SiteOpL<NS> sA, sB;
    OpsShare<NS> sh;
    ops_fetch<NS, MODE>(sh, a);
    cpx<R> z[12];
    hop_all<NS, DAG>(z, a.in, a.Uown, a.Uoth, cb, nb, s, [&] { ops_store<NS, MODE>(sA, sB, sh); });
    const double nrm = hop_epilogue<NS, DAG, MODE, RED>(a, z, cb, s, lane, valid, sA, sB);
    if constexpr (RED) {
        __shared__ double lds[4];
        finish_sum(a.red, block_sum256(nrm, lds));
    }
}

// ===================================================================== t-walk form of the hop
// Workgroup -> (segment, t-chunk) of the t-walk schedule (Sched mode 3).  A segment is 256 / NS
// consecutive sites of a t-slab; the segments form an nyb x (nseg / nyb) grid (y-like, z-like).  The
// workgroups that run at the same time on one XCD take one ty x tz patch of that grid.
__device__ __forceinline__ void tw_tile(int b, int n, const Sched& sc, int nseg, int& seg, int& chunk) {
    if (sc.xcd) {  // hardware dispatches workgroup b to XCD b % 8
        const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
        b = x * q + (x < r ? x : r) + i;
    }
    const int per = sc.ty * sc.tz, nyb = sc.nyb, nzb = nseg / nyb;
    const int intra = b % per, tile = b / per;
    const int npy = nyb / sc.ty, npz = nzb / sc.tz;
    const int py = tile % npy, pz = (tile / npy) % npz;
    chunk = tile / (npy * npz);
    seg = (py * sc.ty + intra % sc.ty) + nyb * (pz * sc.tz + intra / sc.ty);
}

// The t-neighbours of a site have its slab index, so one lane walks its (segment position, s) through
// the slabs t0 .. t0 + tt - 1.  The input column of slab t+1 that the forward t term of slab t loads is,
// projected and multiplied by U_t(x + t)^dag, the backward t term of slab t+2: it is formed once and
// kept for two steps in a lane-private LDS slot (even and odd slabs).  Links are staged per step in LDS; slot 7 holds
// the link of the slab-(t+1) input site that the carry needs instead of the backward t link of slab t.
template <int NS, bool DAG, typename R>
__device__ __forceinline__ void tw_carry(cpx<R>* cw, const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ Uoth,
                                         int cbi, int s) {
    constexpr int SB = DAG ? -1 : +1;
    cpx<R> p[12], h[6], U[9], w[6];
    load_col<NS, false>(p, in, (size_t)cbi, s, 0);
    project<3, SB>(p, h);
#pragma unroll
    for (int k = 0; k < 9; k++) U[k] = Uoth[((size_t)cbi * 4 + 3) * 9 + k];
    link_mul<true>(U, h, w);
#pragma unroll
    for (int j = 0; j < 6; j++) cw[j * 256] = w[j];
}

// XL: the segment holds whole x-lines, and the input columns of the current slab (loaded one step earlier
// as the slab-(t+1) columns) are kept in LDS (xl[12][256]), so the x-direction terms read LDS.
template <int NS, bool DAG, int MODE, bool RED, typename R, bool XL>
__device__ __forceinline__ void tw_step(const HopArgs<R>& a, cpx<R> (*sU)[8][9], const SiteOpL<NS>& sA,
                                        const SiteOpL<NS>& sB, int cb, int s, int lane, cpx<R>* cw, double& nrm,
                                        cpx<R> (*xl)[256]) {
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const int ls = threadIdx.x / NS;
    HOP_FENCE();
    int nb[8];
    neighbours(a.g, cb, a.par, nb);
    // the previous step's reads of sU end at the barrier between this step's link loads and LDS writes
    auto tw_barrier = [] { __syncthreads(); };
    stage_links<NS, R, decltype(tw_barrier), true>(sU, a.Uown, a.Uoth, cb, nb, s, tw_barrier);
    cpx<R> z[12];
#pragma unroll
    for (int j = 0; j < 12; j++) z[j] = {0, 0};
    if constexpr (XL) {  // x +- 1 are sites of this segment: lanes (ls + nb - cb) * NS + s
        const int lf = (ls + nb[0] - cb) * NS + s, lb = (ls + nb[1] - cb) * NS + s;
        cpx<R> p[12], h[6], w[6], U[9];
#pragma unroll
        for (int j = 0; j < 12; j++) p[j] = xl[j][lf];
        project<0, SF>(p, h);
#pragma unroll
        for (int k = 0; k < 9; k++) U[k] = sU[ls][0][k];
        link_mul<false>(U, h, w);
        reconstruct<0, SF>(z, w);
#pragma unroll
        for (int j = 0; j < 12; j++) p[j] = xl[j][lb];
        project<0, SB>(p, h);
#pragma unroll
        for (int k = 0; k < 9; k++) U[k] = sU[ls][4][k];
        link_mul<true>(U, h, w);
        reconstruct<0, SB>(z, w);
    } else {
        hop_mu<NS, DAG, 0>(z, a.in, sU[ls][0], sU[ls][4], nb, s);
    }
    HOP_FENCE();
    hop_mu<NS, DAG, 1>(z, a.in, sU[ls][1], sU[ls][5], nb, s);
    HOP_FENCE();
    hop_mu<NS, DAG, 2>(z, a.in, sU[ls][2], sU[ls][6], nb, s);
    HOP_FENCE();
    {
        // the slab-(t+1) input column: loaded here rather than a step ahead, since a load in flight across
        // the next step's link loads would make their wait (an in-order count) wait for it as well
        cpx<R> p[12], h[6], w[6], U[9];
        load_col<NS, false>(p, a.in, (size_t)nb[6], s, 0);
        if constexpr (XL) {  // every lane has read this slab's columns: keep the next slab's
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 12; j++) xl[j][threadIdx.x] = p[j];
        }
        project<3, SF>(p, h);
#pragma unroll
        for (int k = 0; k < 9; k++) U[k] = sU[ls][3][k];
        link_mul<false>(U, h, w);
        reconstruct<3, SF>(z, w);
#pragma unroll
        for (int j = 0; j < 6; j++) w[j] = cw[j * 256];
        reconstruct<3, SB>(z, w);  // backward t term, carried from two steps back
        project<3, SB>(p, h);
#pragma unroll
        for (int k = 0; k < 9; k++) U[k] = sU[ls][7][k];
        link_mul<true>(U, h, w);   // the backward t term of slab t + 2
#pragma unroll
        for (int j = 0; j < 6; j++) cw[j * 256] = w[j];
    }
    HOP_FENCE();
    nrm += hop_epilogue<NS, DAG, MODE, RED>(a, z, cb, s, lane, true, sA, sB);
    HOP_FENCE();
}

template <int NS, bool DAG, int MODE, bool RED, typename R, bool XL>
__global__ __launch_bounds__(256, 1) void k_hop_tw(const HopArgs<R> a) {
    if (a.done && *a.done != 0.0) return;
    __shared__ cpx<R> sU[256 / NS][8][9];
    __shared__ cpx<R> xl[XL ? 12 : 1][256];  // XL: the current slab's input columns of this segment
    __shared__ SiteOpL<NS> sA, sB;
    {
        OpsShare<NS> sh;
        ops_fetch<NS, MODE>(sh, a);
        ops_store<NS, MODE>(sA, sB, sh);  // published by the first step's barriers
    }
    const int nseg = (int)((size_t)a.g.Vh / a.g.Lt * NS / 256);
    int seg, chunk;
    tw_tile(blockIdx.x, gridDim.x, a.sc, nseg, seg, chunk);
    const int lane = threadIdx.x & 63, s = lane & (NS - 1);
    const int st = a.g.Vh / a.g.Lt;                        // sites per slab
    const int i = seg * (256 / NS) + threadIdx.x / NS;     // slab index of this lane's site
    const int TC = a.sc.tt, t0 = chunk * TC;
    // carried backward t terms, private to each lane: slot t % 2 holds the term of slab t
    __shared__ cpx<R> carry[2][6][256];
    tw_carry<NS, DAG>(&carry[0][0][threadIdx.x], a.in, a.Uoth, i + st * (t0 == 0 ? a.g.Lt - 1 : t0 - 1), s);
    tw_carry<NS, DAG>(&carry[1][0][threadIdx.x], a.in, a.Uoth, i + st * t0, s);
    if constexpr (XL) {  // slab t0's columns; published by the first step's barriers
        cpx<R> p[12];
        load_col<NS, false>(p, a.in, (size_t)(i + st * t0), s, 0);
#pragma unroll
        for (int j = 0; j < 12; j++) xl[j][threadIdx.x] = p[j];
    }
    double nrm = 0.0;
    for (int k = 0; k < TC; k++)
        tw_step<NS, DAG, MODE, RED, R, XL>(a, sU, sA, sB, i + st * (t0 + k), s, lane, &carry[k & 1][0][threadIdx.x],
                                           nrm, xl);
    if constexpr (RED) {
        __shared__ double lds[4];
        finish_sum(a.red, block_sum256(nrm, lds));
    }
}

// ===================================================================== spin-split t-walk form of the hop
// (Sched mode 6.)  The t-walk over whole x-lines with the x neighbours from LDS (mode 5), with two lanes per
// (site, s): the lanes of half H (waves 0-3 for H = 0, waves 4-7 for H = 1 of a 512-lane workgroup) form the
// H-th spin component of every projected half-spinor.  For direction mu that component reads the upper spin
// H and one lower spin of the neighbour column and adds into the same two spins of the output: the lower spin
// 1 - H for x and y, H for z and t.  A lane therefore accumulates the upper spin H throughout, the lower spin
// 1 - H over x and y, and the lower spin H over z and t; between y and z the halves swap their lower-spin
// partial sums through LDS, so every output component collects its eight terms in the order of the unsplit
// hop and the operator is bitwise that of k_hop.  A lane holds half of each column, which leaves registers
// for two waves per SIMD on the same working set of lattice lines as mode 5.

// lower spin that component H of direction MU reads and writes
template <int MU, int H> constexpr int low_spin() { return MU < 2 ? 1 - H : H; }

// h = component H of the projection (1 + S gamma_MU) psi from the upper spin H (up) and the lower spin
// low_spin<MU, H> (dn) of psi; the same operations as project() on that component
template <int MU, int S, int H, typename R>
__device__ __forceinline__ void project_h(const cpx<R> up[3], const cpx<R> dn[3], cpx<R> h[3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cpx<R> b;
        if constexpr (MU == 0) b = cneg(ci(dn[c]));
        else if constexpr (MU == 1) b = H == 0 ? cneg(dn[c]) : dn[c];
        else if constexpr (MU == 2) b = H == 0 ? cneg(ci(dn[c])) : ci(dn[c]);
        else b = dn[c];
        h[c] = S > 0 ? cadd(up[c], b) : csub(up[c], b);
    }
}

// adds component H of (1 + S gamma_MU)-reconstruction of w into the upper spin H (au) and the lower spin
// low_spin<MU, H> (ad); the same operations as reconstruct() on that component
template <int MU, int S, int H, typename R>
__device__ __forceinline__ void reconstruct_h(cpx<R> au[3], cpx<R> ad[3], const cpx<R> w[3]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cpx<R> t;
        if constexpr (MU == 0) t = ci(w[c]);
        else if constexpr (MU == 1) t = H == 0 ? cneg(w[c]) : w[c];
        else if constexpr (MU == 2) t = H == 0 ? ci(w[c]) : cneg(ci(w[c]));
        else t = w[c];
        au[c] = cadd(au[c], w[c]);
        ad[c] = S > 0 ? cadd(ad[c], t) : csub(ad[c], t);
    }
}

// w = U h or U^dag h for one spin component (the arithmetic of link_mul on that component)
template <bool ADJ, typename R>
__device__ __forceinline__ void link_mul3(const cpx<R>* U, const cpx<R> h[3], cpx<R> w[3]) {
    cpx<R> u[9];
#pragma unroll
    for (int k = 0; k < 9; k++) u[k] = U[k];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        cpx<R> a = {0, 0};
#pragma unroll
        for (int k = 0; k < 3; k++) {
            if constexpr (!ADJ) a = cmadd(a, u[3 * r + k], h[k]);
            else a = cjmadd(a, u[3 * k + r], h[k]);
        }
        w[r] = a;
    }
}

// the upper spin H and the lower spin L of column cb (12 NS complex per 4D site, s fastest)
template <int NS, int H, int L, typename R>
__device__ __forceinline__ void load_spins(cpx<R> up[3], cpx<R> dn[3], const cpx<R>* __restrict__ in, size_t cb, int s) {
    const cpx<R>* col = in + cb * 12 * NS + s;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        up[c] = col[(3 * H + c) * NS];
        dn[c] = col[(6 + 3 * L + c) * NS];
    }
}

// one direction MU of component H from global memory: forward term at nb[2 MU], backward at nb[2 MU + 1]
template <int NS, bool DAG, int MU, int H, typename R>
__device__ __forceinline__ void hop_mu_h(cpx<R> au[3], cpx<R> ad[3], const cpx<R>* __restrict__ in, const cpx<R>* Uf,
                                         const cpx<R>* Ub, const int nb[8], int s) {
    constexpr int SF = DAG ? +1 : -1, SB = -SF, L = low_spin<MU, H>();
    {
        cpx<R> up[3], dn[3], h[3], w[3];
        load_spins<NS, H, L>(up, dn, in, (size_t)nb[2 * MU], s);
        project_h<MU, SF, H>(up, dn, h);
        link_mul3<false>(Uf, h, w);
        reconstruct_h<MU, SF, H>(au, ad, w);
    }
    {
        cpx<R> up[3], dn[3], h[3], w[3];
        load_spins<NS, H, L>(up, dn, in, (size_t)nb[2 * MU + 1], s);
        project_h<MU, SB, H>(up, dn, h);
        link_mul3<true>(Ub, h, w);
        reconstruct_h<MU, SB, H>(au, ad, w);
    }
}

// The links of the workgroup's sites staged in LDS by LPS lanes per site (lane li of site ls), slot 7 holding
// U_t of the input site x + t (the t-walk's carry link); more_stores runs between the loads and the LDS writes.
template <int LPS, typename R, typename F>
__device__ __forceinline__ void stage_links_tw(cpx<R> (*sU)[8][9], const cpx<R>* __restrict__ Uown,
                                               const cpx<R>* __restrict__ Uoth, int cb, const int nb[8], int ls, int li,
                                               F more_stores) {
    constexpr int NQ = (72 + LPS - 1) / LPS;
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 v[NQ];
    const int n1 = nb[1], n3 = nb[3], n5 = nb[5], n6 = nb[6];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int e = min(li + q * LPS, 71), l = e / 9, k = e % 9;
        // the input site of backward link l as arithmetic on the four candidates (a select chain or an index
        // into nb[] is turned into a private-memory table)
        const int nbl = (l == 4) * n1 + (l == 5) * n3 + (l == 6) * n5 + (l == 7) * n6;
        const cpx<R>* src = (l < 4) ? Uown + ((size_t)cb * 4 + l) * 9 + k : Uoth + ((size_t)nbl * 4 + (l - 4)) * 9 + k;
        v[q] = *(const v2*)src;
    }
    more_stores();
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int e = li + q * LPS;
        if (e < 72) *(v2*)&sU[ls][e / 9][e % 9] = v[q];
    }
    __syncthreads();
}

// Block-wide sum over 512 lanes (result valid in every thread).
__device__ __forceinline__ double block_sum512(double v, double* lds8) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds8[w] = v;
    __syncthreads();
    return ((lds8[0] + lds8[1]) + (lds8[2] + lds8[3])) + ((lds8[4] + lds8[5]) + (lds8[6] + lds8[7]));
}

// The epilogue of MODE on this lane's share v (v[0..2] the upper spin H, v[3..5] the lower spin H) at (cb, s):
// the operations of hop_epilogue on these components; returns this lane's part of the reduced norm.
template <int NS, bool DAG, int MODE, bool RED, int H, typename R, typename TA, typename TB>
__device__ __forceinline__ double hop_epilogue_h(const HopArgs<R>& a, cpx<R> z[6], int cb, int s, int lane,
                                                 const TA& opA, const TB& opB) {
    const size_t base = (size_t)cb * 12 * NS + s;
    // offset of this lane's j-th component in a column: upper spin H (j < 3), then lower spin H
#define J(j) ((((j) < 3) ? 3 * H + (j) : 3 + 3 * H + (j)) * NS)
    double nrm = 0.0;
    cpx<R> v[6];
    if constexpr (MODE == HM_LIN || MODE == HM_SITE) {
#pragma unroll
        for (int j = 0; j < 6; j++) v[j] = cscale(a.cz, z[j]);
        if (a.aux) {
#pragma unroll
            for (int j = 0; j < 6; j++) {
                cpx<R> t = ld_once(a.aux + base + J(j));
                v[j].x = fma(a.caux, t.x, v[j].x);
                v[j].y = fma(a.caux, t.y, v[j].y);
            }
        }
        if constexpr (MODE == HM_SITE) site_op_half<NS, DAG>(v, opA, s, lane);
    } else if constexpr (MODE == HM_SCHUR_W) {
        site_op_half<NS, false>(z, opA, s, lane);
#pragma unroll
        for (int j = 0; j < 6; j++) {
            cpx<R> t = ld_once(a.aux + base + J(j));
            v[j].x = fma(a.cz, z[j].x, a.caux * t.x);
            v[j].y = fma(a.cz, z[j].y, a.caux * t.y);
        }
    } else if constexpr (MODE == HM_SCHUR_Q) {
        const R alpha = (R)a.scal[SC_ALPHA];
#pragma unroll
        for (int j = 0; j < 6; j++) {
            cpx<R> w = ld_once(a.aux + base + J(j)), r = ld_once(a.aux2 + base + J(j));
            R qx = fma(a.cz, z[j].x, a.caux * w.x), qy = fma(a.cz, z[j].y, a.caux * w.y);
            v[j].x = fma(-alpha, qx, r.x);
            v[j].y = fma(-alpha, qy, r.y);
        }
    } else if constexpr (MODE == HM_DT || MODE == HM_DW) {
        cpx<R> d[6], m[6];
#pragma unroll
        for (int j = 0; j < 6; j++) d[j] = a.self[base + J(j)];
#pragma unroll
        for (int j = 0; j < 6; j++) m[j] = d[j];
        if constexpr (MODE == HM_DT) site_op_half<NS, DAG>(m, opA, s, lane);
#pragma unroll
        for (int j = 0; j < 6; j++) {
            R tx = a.diag * d[j].x - (R)0.5 * z[j].x, ty = a.diag * d[j].y - (R)0.5 * z[j].y;
            if constexpr (MODE == HM_DT) { tx += m[j].x; ty += m[j].y; }
            v[j] = {a.cz * tx, a.cz * ty};
        }
        if (a.aux) {
#pragma unroll
            for (int j = 0; j < 6; j++) {
                cpx<R> t = ld_once(a.aux + base + J(j));
                v[j].x = fma(a.caux, t.x, v[j].x);
                v[j].y = fma(a.caux, t.y, v[j].y);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 6; j++) st_out(a.out + base + J(j), v[j]);
    if constexpr (RED || MODE == HM_SCHUR_W) {
#pragma unroll
        for (int j = 0; j < 6; j++) nrm += (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
    }
    if constexpr (MODE == HM_SCHUR_W) {
        site_op_half<NS, true>(v, opB, s, lane);
#pragma unroll
        for (int j = 0; j < 6; j++) st_out(a.out2 + base + J(j), v[j]);
    }
    return nrm;
#undef J
}

// backward t term of component H of the column of the input site cbi (U_t(cbi)^dag (1 + gamma_t) psi), kept
// in this lane's carry slot (3 complex, stride 512)
template <int NS, bool DAG, int H, typename R>
__device__ __forceinline__ void tws_carry(cpx<R>* cw, const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ Uoth,
                                          int cbi, int s) {
    constexpr int SB = DAG ? -1 : +1;
    cpx<R> up[3], dn[3], h[3], w[3];
    load_spins<NS, H, H>(up, dn, in, (size_t)cbi, s);
    project_h<3, SB, H>(up, dn, h);
    link_mul3<true>(Uoth + ((size_t)cbi * 4 + 3) * 9, h, w);
#pragma unroll
    for (int c = 0; c < 3; c++) cw[c * 512] = w[c];
}

// One t-walk step of component H at (cb, s): the operations of tw_step (XL form) on this lane's share.
template <int NS, bool DAG, int MODE, bool RED, int H, typename R>
__device__ __forceinline__ void tws_step(const HopArgs<R>& a, cpx<R> (*sU)[8][9], const SiteOpL<NS>& sA,
                                         const SiteOpL<NS>& sB, int cb, int s, int lane, int ls, int q, cpx<R>* cw,
                                         double& nrm, cpx<R> (*xl)[256], cpx<R> (*xch)[3][256]) {
    constexpr int SF = DAG ? +1 : -1, SB = -SF;
    HOP_FENCE();
    int nb[8];
    neighbours(a.g, cb, a.par, nb);
    // the previous step's reads of sU end at the barrier between this step's link loads and LDS writes
    stage_links_tw<2 * NS>(sU, a.Uown, a.Uoth, cb, nb, ls, H * NS + s, [] { __syncthreads(); });
    cpx<R> au[3], ad[3];
#pragma unroll
    for (int c = 0; c < 3; c++) { au[c] = {0, 0}; ad[c] = {0, 0}; }
    {   // x +- 1 are sites of this segment: site-lanes (ls + nb - cb) * NS + s of the LDS copy
        constexpr int L = low_spin<0, H>();
        const int lf = (ls + nb[0] - cb) * NS + s, lb = (ls + nb[1] - cb) * NS + s;
        cpx<R> up[3], dn[3], h[3], w[3];
#pragma unroll
        for (int c = 0; c < 3; c++) { up[c] = xl[3 * H + c][lf]; dn[c] = xl[6 + 3 * L + c][lf]; }
        project_h<0, SF, H>(up, dn, h);
        link_mul3<false>(sU[ls][0], h, w);
        reconstruct_h<0, SF, H>(au, ad, w);
#pragma unroll
        for (int c = 0; c < 3; c++) { up[c] = xl[3 * H + c][lb]; dn[c] = xl[6 + 3 * L + c][lb]; }
        project_h<0, SB, H>(up, dn, h);
        link_mul3<true>(sU[ls][4], h, w);
        reconstruct_h<0, SB, H>(au, ad, w);
    }
    HOP_FENCE();
    hop_mu_h<NS, DAG, 1, H>(au, ad, a.in, sU[ls][1], sU[ls][5], nb, s);
    HOP_FENCE();
    // hand the x, y partial of the lower spin 1 - H to the other half and take its partial of the lower spin H;
    // the barrier also ends every lane's reads of this step's x neighbours in xl
#pragma unroll
    for (int c = 0; c < 3; c++) xch[H][c][q] = ad[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; c++) ad[c] = xch[1 - H][c][q];
    HOP_FENCE();
    hop_mu_h<NS, DAG, 2, H>(au, ad, a.in, sU[ls][2], sU[ls][6], nb, s);
    HOP_FENCE();
    {
        cpx<R> up[3], dn[3], h[3], w[3];
        load_spins<NS, H, H>(up, dn, a.in, (size_t)nb[6], s);
#pragma unroll
        for (int c = 0; c < 3; c++) { xl[3 * H + c][q] = up[c]; xl[6 + 3 * H + c][q] = dn[c]; }
        project_h<3, SF, H>(up, dn, h);
        link_mul3<false>(sU[ls][3], h, w);
        reconstruct_h<3, SF, H>(au, ad, w);
#pragma unroll
        for (int c = 0; c < 3; c++) w[c] = cw[c * 512];
        reconstruct_h<3, SB, H>(au, ad, w);  // backward t term, carried from two steps back
        project_h<3, SB, H>(up, dn, h);
        link_mul3<true>(sU[ls][7], h, w);    // the backward t term of slab t + 2
#pragma unroll
        for (int c = 0; c < 3; c++) cw[c * 512] = w[c];
    }
    HOP_FENCE();
    cpx<R> z[6] = {au[0], au[1], au[2], ad[0], ad[1], ad[2]};
    nrm += hop_epilogue_h<NS, DAG, MODE, RED, H>(a, z, cb, s, lane, sA, sB);
    HOP_FENCE();
}

template <int NS, bool DAG, int MODE, bool RED, int H, typename R>
__device__ __forceinline__ double tws_walk(const HopArgs<R>& a, cpx<R> (*sU)[8][9], const SiteOpL<NS>& sA,
                                           const SiteOpL<NS>& sB, cpx<R> (*xl)[256], cpx<R> (*xch)[3][256],
                                           cpx<R> (*carry)[3][512], int i, int st, int t0, int TC, int s, int lane,
                                           int ls, int q) {
    const int tid = threadIdx.x;
    tws_carry<NS, DAG, H>(&carry[0][0][tid], a.in, a.Uoth, i + st * (t0 == 0 ? a.g.Lt - 1 : t0 - 1), s);
    tws_carry<NS, DAG, H>(&carry[1][0][tid], a.in, a.Uoth, i + st * t0, s);
    {   // slab t0's columns (this half's spins); published by the first step's barriers
        cpx<R> up[3], dn[3];
        load_spins<NS, H, H>(up, dn, a.in, (size_t)(i + st * t0), s);
#pragma unroll
        for (int c = 0; c < 3; c++) { xl[3 * H + c][q] = up[c]; xl[6 + 3 * H + c][q] = dn[c]; }
    }
    double nrm = 0.0;
    for (int k = 0; k < TC; k++)
        tws_step<NS, DAG, MODE, RED, H>(a, sU, sA, sB, i + st * (t0 + k), s, lane, ls, q, &carry[k & 1][0][tid], nrm,
                                        xl, xch);
    return nrm;
}

template <int NS, bool DAG, int MODE, bool RED, typename R>
__global__ __launch_bounds__(512, 1) void k_hop_tws(const HopArgs<R> a) {
    if (a.done && *a.done != 0.0) return;
    __shared__ cpx<R> sU[256 / NS][8][9];
    __shared__ cpx<R> xl[12][256];       // the current slab's input columns of this segment
    __shared__ cpx<R> xch[2][3][256];    // lower-spin partial sums handed between the halves
    __shared__ cpx<R> carry[2][3][512];  // carried backward t terms (slot t % 2 for slab t), per lane
    __shared__ SiteOpL<NS> sA, sB;
    {
        OpsShare<NS> sh;
        ops_fetch<NS, MODE>(sh, a);
        ops_store<NS, MODE>(sA, sB, sh);  // published by the first step's barriers
    }
    const int nseg = (int)((size_t)a.g.Vh / a.g.Lt * NS / 256);
    int seg, chunk;
    tw_tile(blockIdx.x, gridDim.x, a.sc, nseg, seg, chunk);
    const int q = threadIdx.x & 255;            // site-lane of the segment
    const int lane = threadIdx.x & 63, s = q % NS, ls = q / NS;
    const int st = a.g.Vh / a.g.Lt;             // sites per slab
    const int i = seg * (256 / NS) + ls;        // slab index of this lane's site
    const int TC = a.sc.tt, t0 = chunk * TC;
    // the two halves run the same sequence of barriers; the branch is uniform per wave
    const double nrm = threadIdx.x < 256
        ? tws_walk<NS, DAG, MODE, RED, 0>(a, sU, sA, sB, xl, xch, carry, i, st, t0, TC, s, lane, ls, q)
        : tws_walk<NS, DAG, MODE, RED, 1>(a, sU, sA, sB, xl, xch, carry, i, st, t0, TC, s, lane, ls, q);
    if constexpr (RED || MODE == HM_SCHUR_W) {
        __shared__ double lds[8];
        finish_sum(a.red, block_sum512(nrm, lds));
    }
}

// ===================================================================== multi-RHS hop
// With H (R = float only) the Krylov fields in, out (not HM_SCHUR_Q), out2 and aux are FP16 columns;
// the residual (aux2 and the output of HM_SCHUR_Q) stays FP32.
template <int NS, bool DAG, int MODE, typename R, bool H>
__global__ __launch_bounds__(256, HOP_WAVES) void k_hop_mr(const HopArgsMR<R> a) {
    const int tid = tile_of(blockIdx.x, gridDim.x, a.sc, a.g) * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int s = lane & (NS - 1);
    int cb = tid / NS;
    const bool valid = cb < a.g.Vh;
    if (!valid) cb = a.g.Vh - 1;
    int nb[8];
    neighbours(a.g, cb, a.par, nb);
    __shared__ cpx<R> sU[256 / NS][8][9];
    __shared__ double lds[4];
    // LDS copies of every system's site-local operators (dynamic LDS: nr for HM_SITE, 2 nr for HM_SCHUR_W),
    // loaded with the links in one round trip
    extern __shared__ double hop_mr_dyn[];
    SiteOpL<NS>* sOps = (SiteOpL<NS>*)hop_mr_dyn;
    constexpr int NOP = MODE == HM_SITE ? 1 : MODE == HM_SCHUR_W ? 2 : 0;
    if constexpr (NOP > 0) {
        SiteOpShare<NS> sh[NRMAX * NOP];
#pragma unroll
        for (int r = 0; r < NRMAX; r++)
            if (r < a.nr) {
                siteop_fetch<NS>(sh[NOP * r], *a.opA[r]);
                if constexpr (NOP == 2) siteop_fetch<NS>(sh[NOP * r + 1], *a.opB[r]);
            }
        stage_links<NS>(sU, a.Uown, a.Uoth, cb, nb, s, [&] {
#pragma unroll
            for (int r = 0; r < NRMAX; r++)
                if (r < a.nr) {
                    siteop_store<NS>(sOps[NOP * r], sh[NOP * r]);
                    if constexpr (NOP == 2) siteop_store<NS>(sOps[NOP * r + 1], sh[NOP * r + 1]);
                }
        });
    } else {
        stage_links<NS>(sU, a.Uown, a.Uoth, cb, nb, s);
    }
    const size_t base = (size_t)cb * 12 * NS + s;
    for (int r = 0; r < a.nr; r++) {
        const double* S = a.scal + r * SC_N;
        if (S[SC_DONE] != 0.0) continue;  // uniform over the grid
        cpx<R> z[12], v[12];
        hop_lds<NS, DAG, R, H>(z, a.in[r], sU[threadIdx.x / NS], nb, s, a.g.Vh);
        double nrm = 0.0;
        if constexpr (MODE == HM_SITE) {
#pragma unroll
            for (int j = 0; j < 12; j++) v[j] = cscale(a.cz, z[j]);
            site_op<NS, DAG>(v, sOps[r], s, lane);
        } else if constexpr (MODE == HM_SCHUR_W) {
            site_op<NS, false>(z, sOps[2 * r], s, lane);
            cpx<R> t[12];
            load_col<NS, H, true>(t, a.aux[r], (size_t)cb, s, a.g.Vh);
#pragma unroll
            for (int j = 0; j < 12; j++) {
                v[j].x = fma(a.cz, z[j].x, a.caux * t[j].x);
                v[j].y = fma(a.cz, z[j].y, a.caux * t[j].y);
            }
        } else {  // HM_SCHUR_Q
            const R alpha = (R)S[SC_ALPHA];
            cpx<R> w[12];
            load_col<NS, H, true>(w, a.aux[r], (size_t)cb, s, a.g.Vh);
            const cpx<R>* aux2 = a.aux2[r] + base;
#pragma unroll
            for (int j = 0; j < 12; j++) {
                cpx<R> rr = ld_once(aux2 + j * NS);
                R qx = fma(a.cz, z[j].x, a.caux * w[j].x), qy = fma(a.cz, z[j].y, a.caux * w[j].y);
                v[j].x = fma(-alpha, qx, rr.x);
                v[j].y = fma(-alpha, qy, rr.y);
            }
        }
        if (valid) store_col<NS, H && MODE != HM_SCHUR_Q>(a.out[r], (size_t)cb, s, a.g.Vh, v);
        if constexpr (MODE != HM_SITE) {
#pragma unroll
            for (int j = 0; j < 12; j++) nrm += (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
            if (!valid) nrm = 0.0;
            if constexpr (MODE == HM_SCHUR_W) {
                site_op<NS, true>(v, sOps[2 * r + 1], s, lane);
                if (valid) store_col<NS, H>(a.out2[r], (size_t)cb, s, a.g.Vh, v);
            }
            const double bs = block_sum256(nrm, lds);
            if (threadIdx.x == 0) a.partials[(size_t)r * a.pstride + blockIdx.x] = bs;
        }
    }
}

// one block per system: finish the reduction of system r (skipped once it is done)
__global__ __launch_bounds__(256) void k_finish_mr(const double* __restrict__ partials, int pstride, unsigned n,
                                                   double* scal, int epi) {
    double* S = scal + blockIdx.x * SC_N;
    if (S[SC_DONE] != 0.0) return;
    finish_partials(partials + (size_t)blockIdx.x * pstride, n, S, 0, epi);
}

// x += alpha p ; p = r + beta p on this block's chunk of XP_U * 256 consecutive elements (one launch covers
// the field, no grid-stride loop): every load of the chunk is issued before the first update, so a thread
// keeps 3 * XP_U elements in flight instead of 3.  NT: nontemporal loads and stores (the launchers use them
// for fields larger than the 256 MB Infinity Cache, where nothing of the five streams is reused before the
// next iteration; 3.03 -> 2.78 ms for FP64 and 1.52 -> 1.37 ms for FP32 at 32^3 x 64, Ns = 16).
template <typename R> constexpr int xp_unroll() { return sizeof(R) == 8 ? 4 : 8; }
template <bool NT, typename R> __device__ __forceinline__ cpx<R> xp_ld(const cpx<R>* q) {
    if constexpr (NT) return {__builtin_nontemporal_load(&q->x), __builtin_nontemporal_load(&q->y)};
    else return *q;
}
template <bool NT, typename R> __device__ __forceinline__ void xp_st(cpx<R>* q, cpx<R> v) {
    if constexpr (NT) {
        __builtin_nontemporal_store(v.x, &q->x);
        __builtin_nontemporal_store(v.y, &q->y);
    } else {
        *q = v;
    }
}
template <typename R, bool NT>
__device__ __forceinline__ void xp_chunk(cpx<R>* __restrict__ x, cpx<R>* __restrict__ p, const cpx<R>* __restrict__ r,
                                         R alpha, R beta, size_t n) {
    constexpr int U = xp_unroll<R>();
    const size_t i0 = (size_t)blockIdx.x * (256 * U) + threadIdx.x;
    cpx<R> pp[U], rr[U], xx[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
        const size_t i = i0 + (size_t)k * 256;
        if (i < n) { pp[k] = xp_ld<NT>(p + i); rr[k] = xp_ld<NT>(r + i); xx[k] = xp_ld<NT>(x + i); }
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
        const size_t i = i0 + (size_t)k * 256;
        if (i < n) {
            cpx<R> a = xx[k], b = pp[k];
            a.x = fma(alpha, b.x, a.x); a.y = fma(alpha, b.y, a.y);
            b.x = fma(beta, b.x, rr[k].x); b.y = fma(beta, b.y, rr[k].y);
            xp_st<NT>(x + i, a);
            xp_st<NT>(p + i, b);
        }
    }
}
// fields above this size take the nontemporal form of the x/p update
constexpr size_t kXpNtBytes = (size_t)256 << 20;
template <typename R> static inline unsigned xp_grid(size_t n) {
    const size_t per = (size_t)256 * xp_unroll<R>();
    return (unsigned)((n + per - 1) / per);
}

template <typename R> struct XpArgs {
    cpx<R>* x[NRMAX];
    cpx<R>* p[NRMAX];
    cpx<R>* r[NRMAX];
};

template <typename R, bool NT>
__global__ __launch_bounds__(256) void k_cg_xp_mr(const XpArgs<R> a, double* scal, size_t n) {
    const int r = blockIdx.y;
    const double* S = scal + r * SC_N;
    if (S[SC_DONEX] != 0.0) return;
    xp_chunk<R, NT>(a.x[r], a.p[r], a.r[r], (R)S[SC_ALPHA], (R)S[SC_BETA], n);
}

// FP16 form: x (FP32) += alpha p ; p (FP16 columns) = r (FP32) + beta p; one thread per (cb, s).  The stores
// are nontemporal; NT: the loads too (fields above the Infinity Cache, as in xp_chunk).
template <int NS, bool NT>
__global__ __launch_bounds__(256) void k_cg_xp_mr_h(const XpArgs<float> a, double* scal, int Vh) {
    const int r = blockIdx.y;
    const double* S = scal + r * SC_N;
    if (S[SC_DONEX] != 0.0) return;
    const float alpha = (float)S[SC_ALPHA], beta = (float)S[SC_BETA];
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;  // one (cb, s) column per thread, no loop
    if (t < (size_t)Vh * NS) {
        const size_t cb = t / NS;
        const int s = (int)(t % NS);
        cpx<float> p[12], x[12], q[12];
        load_h<NS, NT>(p, a.p[r], cb, s, Vh);
        load_col<NS, false, NT>(x, a.x[r], cb, s, Vh);
        load_col<NS, false, NT>(q, a.r[r], cb, s, Vh);
#pragma unroll
        for (int j = 0; j < 12; j++) {
            x[j].x = fmaf(alpha, p[j].x, x[j].x); x[j].y = fmaf(alpha, p[j].y, x[j].y);
            p[j].x = fmaf(beta, p[j].x, q[j].x);  p[j].y = fmaf(beta, p[j].y, q[j].y);
        }
        store_col<NS, false>(a.x[r], cb, s, Vh, x);
        store_h<NS>(a.p[r], cb, s, Vh, p);
    }
}

// FP32 half field -> FP16 columns
template <int NS>
__global__ __launch_bounds__(256) void k_f2h(const cpx<float>* __restrict__ in, void* __restrict__ out, int Vh) {
    for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < (size_t)Vh * NS; t += (size_t)gridDim.x * 256) {
        const size_t cb = t / NS;
        const int s = (int)(t % NS);
        cpx<float> v[12];
        load_col<NS, false>(v, in, cb, s, Vh);
        store_h<NS>(out, cb, s, Vh, v);
    }
}

// FP16 columns -> FP64 half field (diagnostics and tests)
template <int NS>
__global__ __launch_bounds__(256) void k_h2d(const void* __restrict__ in, cd* __restrict__ out, int Vh) {
    for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < (size_t)Vh * NS; t += (size_t)gridDim.x * 256) {
        const size_t cb = t / NS;
        const int s = (int)(t % NS);
        cpx<float> v[12];
        load_h<NS>(v, in, cb, s, Vh);
        cd* dst = out + cb * 12 * NS + s;
#pragma unroll
        for (int j = 0; j < 12; j++) dst[j * NS] = {(double)v[j].x, (double)v[j].y};
    }
}

// After the x/p update of an iteration: count it if it was applied, then let SC_DONEX catch up with SC_DONE
// (the update of the converging iteration itself is applied; later ones are skipped).
__global__ void k_sync_done(double* scal, int nr) {
    if (threadIdx.x < nr) {
        double* S = scal + threadIdx.x * SC_N;
        if (S[SC_DONEX] == 0.0) S[SC_ITERS] += 1.0;
        S[SC_DONEX] = S[SC_DONE];
    }
}

// ===================================================================== site-local op only
template <int NS, bool DAG, typename R>
__global__ __launch_bounds__(256) void k_site(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                              const SiteOp* __restrict__ op, int Vh) {
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int s = lane & (NS - 1);
    int cb = tid / NS;
    const bool valid = cb < Vh;
    if (!valid) cb = Vh - 1;
    const size_t base = (size_t)cb * 12 * NS + s;
    cpx<R> v[12];
#pragma unroll
    for (int j = 0; j < 12; j++) v[j] = in[base + j * NS];
    site_op<NS, DAG>(v, *op, s, lane);
    if (valid) {
#pragma unroll
        for (int j = 0; j < 12; j++) out[base + j * NS] = v[j];
    }
}

// ===================================================================== BLAS-1
// CG step after the residual update: x += alpha p ; p = r + beta p   (alpha, beta on device; skipped once
// the update of the converging iteration has been applied)
template <typename R, bool NT>
__global__ __launch_bounds__(256) void k_cg_xp(cpx<R>* __restrict__ x, cpx<R>* __restrict__ p,
                                               const cpx<R>* __restrict__ r, const double* __restrict__ scal,
                                               size_t n) {
    if (scal[SC_DONEX] != 0.0) return;
    xp_chunk<R, NT>(x, p, r, (R)scal[SC_ALPHA], (R)scal[SC_BETA], n);
}

// y = a*x + b*y, with an optional |y|^2 reduction
template <typename R, bool RED>
__global__ __launch_bounds__(256) void k_axpby(R a, const cpx<R>* __restrict__ x, R b, cpx<R>* __restrict__ y,
                                               size_t n, Red red) {
    double nrm = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        cpx<R> xx = x ? x[i] : cpx<R>{0, 0}, yy = y[i];
        yy.x = fma(a, xx.x, b * yy.x); yy.y = fma(a, xx.y, b * yy.y);
        y[i] = yy;
        if constexpr (RED) nrm += (double)yy.x * yy.x + (double)yy.y * yy.y;
    }
    if constexpr (RED) {
        __shared__ double lds[4];
        finish_sum(red, block_sum256(nrm, lds));
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_norm2(const cpx<R>* __restrict__ x, size_t n, Red red) {
    double nrm = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        cpx<R> xx = x[i];
        nrm += (double)xx.x * xx.x + (double)xx.y * xx.y;
    }
    __shared__ double lds[4];
    finish_sum(red, block_sum256(nrm, lds));
}

// precision conversion: out = (To) in
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_convert(const cpx<Ti>* __restrict__ in, cpx<To>* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        cpx<Ti> v = in[i];
        out[i] = {(To)v.x, (To)v.y};
    }
}

// x_hi += (double) x_lo
template <typename R>
__global__ __launch_bounds__(256) void k_accum_lo(cd* __restrict__ xhi, const cpx<R>* __restrict__ xlo, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        cpx<R> v = xlo[i];
        cd h = xhi[i];
        xhi[i] = {h.x + (double)v.x, h.y + (double)v.y};
    }
}

// complex dot products <v_i, y> = sum conj(v_i) y for i < nv (nv <= 9): partials[2i][blk] (re), [2i+1][blk] (im)
struct DotArgs {
    const cd* v[9];
    int nv;
};
__global__ __launch_bounds__(256) void k_mdot(const DotArgs a, const cd* __restrict__ y, size_t n, double* partials,
                                              int pstride) {
    double re[9], im[9];
#pragma unroll
    for (int i = 0; i < 9; i++) { re[i] = 0; im[i] = 0; }
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
        const cd yy = y[k];
#pragma unroll
        for (int i = 0; i < 9; i++)
            if (i < a.nv) {
                const cd vv = a.v[i][k];
                re[i] = fma(vv.x, yy.x, fma(vv.y, yy.y, re[i]));
                im[i] = fma(vv.x, yy.y, fma(-vv.y, yy.x, im[i]));
            }
    }
    __shared__ double lds[4];
    for (int i = 0; i < a.nv; i++) {
        const double r = block_sum256(re[i], lds);
        const double m = block_sum256(im[i], lds);
        if (threadIdx.x == 0) {
            partials[(size_t)(2 * i) * pstride + blockIdx.x] = r;
            partials[(size_t)(2 * i + 1) * pstride + blockIdx.x] = m;
        }
    }
}

// y += sum_i c_i v_i (complex c_i, nv <= 9)
struct AxpyArgs {
    const cd* v[9];
    double cr[9], ci[9];
    int nv;
};
__global__ __launch_bounds__(256) void k_maxpy(const AxpyArgs a, cd* __restrict__ y, size_t n) {
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
        cd yy = y[k];
        for (int i = 0; i < a.nv; i++) {
            const cd vv = a.v[i][k];
            yy.x = fma(a.cr[i], vv.x, fma(-a.ci[i], vv.y, yy.x));
            yy.y = fma(a.cr[i], vv.y, fma(a.ci[i], vv.x, yy.y));
        }
        y[k] = yy;
    }
}

__global__ void k_finish_many(const double* __restrict__ partials, int pstride, unsigned n, double* out) {
    // block b sums partials[b * pstride .. + n) into out[b]
    __shared__ double lds[4];
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < n; i += 256) s += partials[(size_t)blockIdx.x * pstride + i];
    s = block_sum256(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ===================================================================== boundary kernels
// canonical index of (s, lex site, j): ((s * V + lex) * 12 + j)
__device__ __forceinline__ void cb_to_lex(const Geom& g, int cb, int par, int& lex) {
    int xh = cb % g.Lxh;
    int r = cb / g.Lxh;
    int y = r % g.Ly; r /= g.Ly;
    int z = r % g.Lz;
    int t = r / g.Lz;
    int x = 2 * xh + ((y + z + t + par) & 1);
    lex = x + g.Lx * (y + g.Ly * (z + g.Lz * t));
}

// canonical 5D (complex128) <-> internal half field of parity par.  One thread per (cb, j, s).
// refl != 0 applies R5 gamma_5 on the way: half(s) = gamma_5 canon(Ns - 1 - s), gamma_5 = diag(1, 1, -1, -1).
template <typename R>
__global__ __launch_bounds__(256) void k_pack5(const cd* __restrict__ canon, cpx<R>* __restrict__ half, Geom g,
                                               int par, int Ns, int refl) {
    const size_t n = (size_t)g.Vh * 12 * Ns;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        int s = (int)(i % Ns);
        int j = (int)((i / Ns) % 12);
        int cb = (int)(i / ((size_t)12 * Ns));
        int lex;
        cb_to_lex(g, cb, par, lex);
        int sc = refl ? Ns - 1 - s : s;
        cd v = canon[((size_t)sc * (2 * (size_t)g.Vh) + lex) * 12 + j];
        double sg = (refl && j >= 6) ? -1.0 : 1.0;
        half[i] = {(R)(sg * v.x), (R)(sg * v.y)};
    }
}

// refl != 0 applies gamma_5 R5 on the way: canon(Ns - 1 - s) = gamma_5 half(s).
template <typename R>
__global__ __launch_bounds__(256) void k_unpack5(const cpx<R>* __restrict__ half, cd* __restrict__ canon, Geom g,
                                                 int par, int Ns, int refl) {
    const size_t n = (size_t)g.Vh * 12 * Ns;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        int s = (int)(i % Ns);
        int j = (int)((i / Ns) % 12);
        int cb = (int)(i / ((size_t)12 * Ns));
        int lex;
        cb_to_lex(g, cb, par, lex);
        cpx<R> v = half[i];
        int sc = refl ? Ns - 1 - s : s;
        double sg = (refl && j >= 6) ? -1.0 : 1.0;
        canon[((size_t)sc * (2 * (size_t)g.Vh) + lex) * 12 + j] = {sg * (double)v.x, sg * (double)v.y};
    }
}

// links: canonical [lex][mu][3][3] -> packed [par][cb][mu][9], t-boundary phase folded into U_t(x_t = Lt-1)
template <typename R>
__global__ __launch_bounds__(256) void k_pack_links(const cd* __restrict__ U, cpx<R>* __restrict__ Up, Geom g,
                                                    int par, double tbc) {
    const size_t n = (size_t)g.Vh * 36;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        int k = (int)(i % 9);
        int mu = (int)((i / 9) % 4);
        int cb = (int)(i / 36);
        int lex;
        cb_to_lex(g, cb, par, lex);
        cd v = U[((size_t)lex * 4 + mu) * 9 + k];
        int t = lex / (g.Lx * g.Ly * g.Lz);
        if (mu == 3 && t == g.Lt - 1) { v.x *= tbc; v.y *= tbc; }
        Up[i] = {(R)v.x, (R)v.y};
    }
}

// EOFA source: c_s = coef[s] * P_chir phi at every site of parity par (coef[s] = chir * Om_{Ns-1-s},
// i.e. c = R5 gamma_5 (Om (x) P_chir phi)).  One thread per (cb, j, s).
__global__ __launch_bounds__(256) void k_source(const cd* __restrict__ phi, cd* __restrict__ half, Geom g, int par,
                                                int Ns, int chir, const double* __restrict__ coef) {
    const size_t n = (size_t)g.Vh * 12 * Ns;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        int s = (int)(i % Ns);
        int j = (int)((i / Ns) % 12);
        int cb = (int)(i / ((size_t)12 * Ns));
        int lex;
        cb_to_lex(g, cb, par, lex);
        int spin = j / 3;
        bool keep = (chir > 0) ? (spin < 2) : (spin >= 2);
        cd v = phi[(size_t)lex * 12 + j];
        double c = keep ? coef[s] : 0.0;
        half[i] = {c * v.x, c * v.y};
    }
}

// EOFA combine: out = P_chir phi + ck * sum_s Om_s P_chir x_s on the sites of parity par, and the
// partial sums of Re phi^dag out.  One thread per (cb, j).
__global__ __launch_bounds__(256) void k_combine(const cd* __restrict__ phi, const cd* __restrict__ xh, cd* __restrict__ out,
                                                 Geom g, int par, int Ns, int chir, double ck,
                                                 const double* __restrict__ Om, int accumulate, Red red) {
    const size_t n = (size_t)g.Vh * 12;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        int j = (int)(i % 12);
        int cb = (int)(i / 12);
        int lex;
        cb_to_lex(g, cb, par, lex);
        int spin = j / 3;
        bool keep = (chir > 0) ? (spin < 2) : (spin >= 2);
        cd ph = phi[(size_t)lex * 12 + j];
        cd o = {0.0, 0.0};
        if (keep) {
            double sx = 0.0, sy = 0.0;
            const cd* src = xh + ((size_t)cb * 12 + j) * Ns;
            for (int s = 0; s < Ns; s++) { sx = fma(Om[s], src[s].x, sx); sy = fma(Om[s], src[s].y, sy); }
            o = {ph.x + ck * sx, ph.y + ck * sy};
        }
        cd* dst = out + (size_t)lex * 12 + j;
        if (accumulate) { cd t = *dst; o.x += t.x; o.y += t.y; }
        *dst = o;
        // Re phi^dag (this action's part only)
        if (keep) acc += ph.x * o.x + ph.y * o.y;
    }
    __shared__ double lds[4];
    finish_sum(red, block_sum256(acc, lds));
}

// dst = 0 / dst = src over n doubles (kernels rather than memset / memcpy nodes, so that a caller may capture
// them in a graph)
__global__ __launch_bounds__(256) void k_fill0(double* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = 0.0;
}
__global__ __launch_bounds__(256) void k_copy(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// Heat-bath combination: phi = a0 P_chir eta + sum_l coef[l] out[l] (+ phi when accumulate) at every site, with
// the partial sums of |P_chir eta|^2.  One thread per (site, component) of the canonical 4D field.
__global__ __launch_bounds__(256) void k_hb_combine(const cd* __restrict__ eta, cd* __restrict__ phi, const HbTerms t,
                                                    size_t n, int chir, int accumulate, Red red) {
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const int spin = (int)((i % 12) / 3);
        const bool keep = (chir > 0) ? (spin < 2) : (spin >= 2);
        const cd e = eta[i];
        cd v = keep ? cd{t.a0 * e.x, t.a0 * e.y} : cd{0.0, 0.0};
        for (int l = 0; l < t.n; l++) {
            const cd o = t.out[l][i];
            v.x = fma(t.coef[l], o.x, v.x);
            v.y = fma(t.coef[l], o.y, v.y);
        }
        if (accumulate) { const cd p = phi[i]; v.x += p.x; v.y += p.y; }
        phi[i] = v;
        if (keep) acc += e.x * e.x + e.y * e.y;
    }
    __shared__ double lds[4];
    finish_sum(red, block_sum256(acc, lds));
}

struct Vec64 {
    double v[64];
};
__global__ void k_set_vec(double* dst, int n, const Vec64 vals) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = vals.v[threadIdx.x];
}

__global__ void k_scal_set(double* S, int s0, double v0, int s1, double v1, int s2, double v2) {
    if (threadIdx.x == 0) {
        if (s0 >= 0) S[s0] = v0;
        if (s1 >= 0) S[s1] = v1;
        if (s2 >= 0) S[s2] = v2;
    }
}

__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ partials, unsigned n, double* S, int slot,
                                                int epi) {
    finish_partials(partials, n, S, slot, epi);
}

// ===================================================================== launchers
static inline void finish(const Red& r, unsigned nblocks, hipStream_t st) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, st, r.partials, nblocks, r.scal, r.slot, r.epi);
}

hipError_t launch_finish(const Red& r, unsigned nblocks, hipStream_t st) {
    finish(r, nblocks, st);
    return hipGetLastError();
}

static inline int nblk(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b > 4096 ? 4096 : b);
}

hipError_t launch_mdot(const cd* const* v, int nv, const cd* y, size_t n, double* partials, int pstride, double* out,
                       hipStream_t st) {
    if (nv < 1 || nv > 9) return hipErrorInvalidValue;
    DotArgs a{};
    for (int i = 0; i < nv; i++) a.v[i] = v[i];
    a.nv = nv;
    const int grid = nblk(n) > 1024 ? 1024 : nblk(n);
    if (grid > pstride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mdot, dim3(grid), dim3(256), 0, st, a, y, n, partials, pstride);
    hipLaunchKernelGGL(k_finish_many, dim3(2 * nv), dim3(256), 0, st, partials, pstride, (unsigned)grid, out);
    return hipGetLastError();
}

hipError_t launch_maxpy(const cd* const* v, const double* cr, const double* ci, int nv, cd* y, size_t n, hipStream_t st) {
    if (nv < 0 || nv > 9) return hipErrorInvalidValue;
    if (nv == 0) return hipSuccess;
    AxpyArgs a{};
    for (int i = 0; i < nv; i++) { a.v[i] = v[i]; a.cr[i] = cr[i]; a.ci[i] = ci[i]; }
    a.nv = nv;
    hipLaunchKernelGGL(k_maxpy, dim3(nblk(n)), dim3(256), 0, st, a, y, n);
    return hipGetLastError();
}

#define NS_SWITCH(NSV, ...)                                            \
    switch (NSV) {                                                     \
    case 4: { constexpr int NS = 4; __VA_ARGS__; break; }              \
    case 8: { constexpr int NS = 8; __VA_ARGS__; break; }              \
    case 16: { constexpr int NS = 16; __VA_ARGS__; break; }            \
    case 32: { constexpr int NS = 32; __VA_ARGS__; break; }            \
    default: return hipErrorInvalidValue;                              \
    }

// Whether schedule sc (mode 3 or 5) fits the lattice and Ns; the t-walk grid size when it does, else 0.
int tw_grid(const Geom& g, int Ns, const Sched& sc) {
    if ((sc.mode != 3 && sc.mode != 5 && sc.mode != 6) || Ns < 8) return 0;
    if (sc.mode == 6 && Ns != 16) return 0;  // the spin-split form is built for Ns = 16
    if (sc.mode >= 5 && (256 / Ns) % g.Lxh) return 0;  // the segment must hold whole x-lines
    const long slab = (long)g.Vh / g.Lt;
    if ((slab * Ns) % 256 != 0) return 0;
    const long nseg = slab * Ns / 256;
    if (sc.tt < 2 || sc.tt % 2 || g.Lt % sc.tt || sc.nyb < 1 || nseg % sc.nyb) return 0;
    if (sc.ty < 1 || sc.tz < 1 || sc.nyb % sc.ty || (nseg / sc.nyb) % sc.tz) return 0;
    if (sc.ord < 0 || sc.ord > 64) return 0;  // static LDS of the t-walk is at most 84 KB
    return (int)(nseg * (g.Lt / sc.tt));
}

// LDS that a launch of kern may reserve on top of its static LDS (gfx950: 160 KB per workgroup).
template <typename K> static size_t lds_room(K kern) {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, (const void*)kern) != hipSuccess) return 0;
    return at.sharedSizeBytes < 160 * 1024 ? 160 * 1024 - at.sharedSizeBytes : 0;
}

template <typename R>
hipError_t launch_hop(int Ns, bool dag, int mode, bool red, const HopArgs<R>& a, hipStream_t st) {
    const size_t nthreads = (size_t)a.g.Vh * Ns;
    const bool tw = a.sc.mode == 3 || a.sc.mode == 5 || a.sc.mode == 6;
    const int grid = tw ? tw_grid(a.g, Ns, a.sc) : (int)((nthreads + 255) / 256);
    if (grid <= 0) return hipErrorInvalidValue;
    const size_t pad = tw ? (size_t)a.sc.ord * 1024 : 0;  // LDS reserved to cap workgroups per CU
#define HOP_L(D, M, RD)                                                                                  \
    do {                                                                                                 \
        if constexpr (NS == 16) {                                                                        \
            if (tw && a.sc.mode == 6) {                                                                  \
                hipLaunchKernelGGL((k_hop_tws<NS, D, M, RD, R>), dim3(grid), dim3(512), 0, st, a);          \
                break;                                                                                   \
            }                                                                                            \
        }                                                                                                \
        if constexpr (NS >= 8) {                                                                         \
            if (tw && a.sc.mode == 5) {                                                                  \
                static const size_t room = lds_room(k_hop_tw<NS, D, M, RD, R, true>);                    \
                hipLaunchKernelGGL((k_hop_tw<NS, D, M, RD, R, true>), dim3(grid), dim3(256),              \
                                   pad < room ? pad : room, st, a);                                      \
                break;                                                                                   \
            }                                                                                            \
            if (tw) {                                                                                    \
                static const size_t room = lds_room(k_hop_tw<NS, D, M, RD, R, false>);                   \
                hipLaunchKernelGGL((k_hop_tw<NS, D, M, RD, R, false>), dim3(grid), dim3(256),             \
                                   pad < room ? pad : room, st, a);                                      \
                break;                                                                                   \
            }                                                                                            \
        }                                                                                                \
        hipLaunchKernelGGL((k_hop<NS, D, M, RD, R>), dim3(grid), dim3(256), 0, st, a);                  \
    } while (0)
#define HOP_MODES(D)                                                                        \
    switch (mode) {                                                                         \
    case HM_LIN: if (red) HOP_L(D, HM_LIN, true); else HOP_L(D, HM_LIN, false); break;     \
    case HM_SITE: if (red) HOP_L(D, HM_SITE, true); else HOP_L(D, HM_SITE, false); break;  \
    case HM_SCHUR_W: HOP_L(D, HM_SCHUR_W, true); break;                                     \
    case HM_SCHUR_Q: HOP_L(D, HM_SCHUR_Q, true); break;                                     \
    case HM_DT: if (red) HOP_L(D, HM_DT, true); else HOP_L(D, HM_DT, false); break;        \
    case HM_DW: HOP_L(D, HM_DW, false); break;                                              \
    default: return hipErrorInvalidValue;                                                   \
    }
    NS_SWITCH(Ns, if (dag) { HOP_MODES(true) } else { HOP_MODES(false) });
#undef HOP_MODES
#undef HOP_L
    if (red || mode == HM_SCHUR_W || mode == HM_SCHUR_Q) finish(a.red, (unsigned)grid, st);
    return hipGetLastError();
}
template hipError_t launch_hop<double>(int, bool, int, bool, const HopArgs<double>&, hipStream_t);
template hipError_t launch_hop<float>(int, bool, int, bool, const HopArgs<float>&, hipStream_t);

template <typename R>
hipError_t launch_hop_mr(int Ns, bool dag, int mode, const HopArgsMR<R>& a, hipStream_t st, bool half) {
    if (a.nr < 1 || a.nr > NRMAX) return hipErrorInvalidValue;
    if (half && sizeof(R) != 4) return hipErrorInvalidValue;
    const int grid = (int)(((size_t)a.g.Vh * Ns + 255) / 256);
    if (grid > a.pstride) return hipErrorInvalidValue;
#define MR_L(D, M)                                                                                       \
    do {                                                                                                 \
        const size_t ops = (size_t)a.nr * (M == HM_SITE ? 1 : M == HM_SCHUR_W ? 2 : 0) * sizeof(SiteOpL<NS>); \
        if constexpr (sizeof(R) == 4) {                                                                  \
            if (half) { hipLaunchKernelGGL((k_hop_mr<NS, D, M, R, true>), dim3(grid), dim3(256), ops, st, a); break; } \
        }                                                                                                \
        hipLaunchKernelGGL((k_hop_mr<NS, D, M, R, false>), dim3(grid), dim3(256), ops, st, a);          \
    } while (0)
#define MR_MODES(D)                                            \
    switch (mode) {                                            \
    case HM_SITE: MR_L(D, HM_SITE); break;                     \
    case HM_SCHUR_W: MR_L(D, HM_SCHUR_W); break;               \
    case HM_SCHUR_Q: MR_L(D, HM_SCHUR_Q); break;               \
    default: return hipErrorInvalidValue;                      \
    }
    switch (Ns) {
    case 8: { constexpr int NS = 8; if (dag) { MR_MODES(true) } else { MR_MODES(false) } break; }
    case 16: { constexpr int NS = 16; if (dag) { MR_MODES(true) } else { MR_MODES(false) } break; }
    case 32: { constexpr int NS = 32; if (dag) { MR_MODES(true) } else { MR_MODES(false) } break; }
    default: return hipErrorInvalidValue;
    }
#undef MR_MODES
#undef MR_L
    if (mode != HM_SITE)
        hipLaunchKernelGGL(k_finish_mr, dim3(a.nr), dim3(256), 0, st, a.partials, a.pstride, (unsigned)grid, a.scal,
                           a.epi);
    return hipGetLastError();
}
template hipError_t launch_hop_mr<double>(int, bool, int, const HopArgsMR<double>&, hipStream_t, bool);
template hipError_t launch_hop_mr<float>(int, bool, int, const HopArgsMR<float>&, hipStream_t, bool);

hipError_t launch_cg_xp_mr_h(int Ns, int nr, cpx<float>* const* x, void* const* p, cpx<float>* const* r, double* scal,
                             int Vh, hipStream_t st) {
    if (nr < 1 || nr > NRMAX) return hipErrorInvalidValue;
    XpArgs<float> a{};
    for (int i = 0; i < nr; i++) { a.x[i] = x[i]; a.p[i] = (cpx<float>*)p[i]; a.r[i] = r[i]; }
    const unsigned gx = (unsigned)(((size_t)Vh * Ns + 255) / 256);
    const bool nt = (size_t)Vh * Ns * 12 * sizeof(cpx<float>) > kXpNtBytes;  // the FP32 x and r fields
#define XPH(NS_)                                                                                                   \
    if (nt) hipLaunchKernelGGL((k_cg_xp_mr_h<NS_, true>), dim3(gx, nr), dim3(256), 0, st, a, scal, Vh);           \
    else hipLaunchKernelGGL((k_cg_xp_mr_h<NS_, false>), dim3(gx, nr), dim3(256), 0, st, a, scal, Vh);
    switch (Ns) {
    case 8: XPH(8) break;
    case 16: XPH(16) break;
    case 32: XPH(32) break;
    default: return hipErrorInvalidValue;
    }
#undef XPH
    hipLaunchKernelGGL(k_sync_done, dim3(1), dim3(64), 0, st, scal, nr);
    return hipGetLastError();
}

hipError_t launch_f2h(int Ns, const cpx<float>* in, void* out, int Vh, hipStream_t st) {
    const int g = nblk((size_t)Vh * Ns);
    NS_SWITCH(Ns, hipLaunchKernelGGL((k_f2h<NS>), dim3(g), dim3(256), 0, st, in, out, Vh));
    return hipGetLastError();
}

hipError_t launch_h2d(int Ns, const void* in, cd* out, int Vh, hipStream_t st) {
    const int g = nblk((size_t)Vh * Ns);
    NS_SWITCH(Ns, hipLaunchKernelGGL((k_h2d<NS>), dim3(g), dim3(256), 0, st, in, out, Vh));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_xp_mr(int nr, cpx<R>* const* x, cpx<R>* const* p, cpx<R>* const* r, double* scal, size_t n,
                           hipStream_t st) {
    if (nr < 1 || nr > NRMAX) return hipErrorInvalidValue;
    XpArgs<R> a{};
    for (int i = 0; i < nr; i++) { a.x[i] = x[i]; a.p[i] = p[i]; a.r[i] = r[i]; }
    if (n * sizeof(cpx<R>) > kXpNtBytes)
        hipLaunchKernelGGL((k_cg_xp_mr<R, true>), dim3(xp_grid<R>(n), nr), dim3(256), 0, st, a, scal, n);
    else
        hipLaunchKernelGGL((k_cg_xp_mr<R, false>), dim3(xp_grid<R>(n), nr), dim3(256), 0, st, a, scal, n);
    hipLaunchKernelGGL(k_sync_done, dim3(1), dim3(64), 0, st, scal, nr);
    return hipGetLastError();
}
template hipError_t launch_cg_xp_mr<double>(int, cd* const*, cd* const*, cd* const*, double*, size_t, hipStream_t);
template hipError_t launch_cg_xp_mr<float>(int, cpx<float>* const*, cpx<float>* const*, cpx<float>* const*, double*,
                                           size_t, hipStream_t);

template <typename R>
hipError_t launch_site(int Ns, bool dag, const cpx<R>* in, cpx<R>* out, const SiteOp* op, int Vh, hipStream_t st) {
    const int grid = (int)(((size_t)Vh * Ns + 255) / 256);
    NS_SWITCH(Ns, if (dag) hipLaunchKernelGGL((k_site<NS, true, R>), dim3(grid), dim3(256), 0, st, in, out, op, Vh);
              else hipLaunchKernelGGL((k_site<NS, false, R>), dim3(grid), dim3(256), 0, st, in, out, op, Vh));
    return hipGetLastError();
}
template hipError_t launch_site<double>(int, bool, const cd*, cd*, const SiteOp*, int, hipStream_t);
template hipError_t launch_site<float>(int, bool, const cpx<float>*, cpx<float>*, const SiteOp*, int, hipStream_t);

template <typename R>
hipError_t launch_cg_xp(cpx<R>* x, cpx<R>* p, const cpx<R>* r, double* scal, size_t n, hipStream_t st) {
    if (n * sizeof(cpx<R>) > kXpNtBytes)
        hipLaunchKernelGGL((k_cg_xp<R, true>), dim3(xp_grid<R>(n)), dim3(256), 0, st, x, p, r, scal, n);
    else
        hipLaunchKernelGGL((k_cg_xp<R, false>), dim3(xp_grid<R>(n)), dim3(256), 0, st, x, p, r, scal, n);
    return hipGetLastError();
}
template hipError_t launch_cg_xp<double>(cd*, cd*, const cd*, double*, size_t, hipStream_t);
template hipError_t launch_cg_xp<float>(cpx<float>*, cpx<float>*, const cpx<float>*, double*, size_t, hipStream_t);

hipError_t launch_sync_done(double* scal, int nr, hipStream_t st) {
    hipLaunchKernelGGL(k_sync_done, dim3(1), dim3(64), 0, st, scal, nr);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_axpby(R a, const cpx<R>* x, R b, cpx<R>* y, size_t n, const Red* red, hipStream_t st) {
    if (red) {
        hipLaunchKernelGGL((k_axpby<R, true>), dim3(nblk(n)), dim3(256), 0, st, a, x, b, y, n, *red);
        finish(*red, (unsigned)nblk(n), st);
    } else hipLaunchKernelGGL((k_axpby<R, false>), dim3(nblk(n)), dim3(256), 0, st, a, x, b, y, n, Red{});
    return hipGetLastError();
}
template hipError_t launch_axpby<double>(double, const cd*, double, cd*, size_t, const Red*, hipStream_t);
template hipError_t launch_axpby<float>(float, const cpx<float>*, float, cpx<float>*, size_t, const Red*, hipStream_t);

template <typename R>
hipError_t launch_norm2(const cpx<R>* x, size_t n, const Red& red, hipStream_t st) {
    hipLaunchKernelGGL((k_norm2<R>), dim3(nblk(n)), dim3(256), 0, st, x, n, red);
    finish(red, (unsigned)nblk(n), st);
    return hipGetLastError();
}
template hipError_t launch_norm2<double>(const cd*, size_t, const Red&, hipStream_t);
template hipError_t launch_norm2<float>(const cpx<float>*, size_t, const Red&, hipStream_t);

hipError_t launch_set_vec(double* dst, int n, const double* host_vals, hipStream_t st) {
    if (n < 0 || n > 64) return hipErrorInvalidValue;
    Vec64 v{};
    for (int i = 0; i < n; i++) v.v[i] = host_vals[i];
    hipLaunchKernelGGL(k_set_vec, dim3(1), dim3(64), 0, st, dst, n, v);
    return hipGetLastError();
}

hipError_t launch_hb_combine(const cd* eta, cd* phi, const HbTerms& t, size_t n, int chir, int accumulate,
                             const Red& red, hipStream_t st) {
    if (t.n < 0 || t.n > HB_MAXTERMS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_hb_combine, dim3(nblk(n)), dim3(256), 0, st, eta, phi, t, n, chir, accumulate, red);
    finish(red, (unsigned)nblk(n), st);
    return hipGetLastError();
}

hipError_t launch_fill0(void* dst, size_t bytes, hipStream_t st) {
    if (bytes % sizeof(double)) return hipErrorInvalidValue;
    const size_t n = bytes / sizeof(double);
    if (n) hipLaunchKernelGGL(k_fill0, dim3(nblk(n)), dim3(256), 0, st, (double*)dst, n);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes % sizeof(double)) return hipErrorInvalidValue;
    const size_t n = bytes / sizeof(double);
    if (n) hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(256), 0, st, (double*)dst, (const double*)src, n);
    return hipGetLastError();
}

hipError_t launch_set_block(double* dst, size_t n, const double* host_vals, hipStream_t st) {
    for (size_t i = 0; i < n; i += 64) {
        const int m = (int)std::min<size_t>(64, n - i);
        hipError_t e = launch_set_vec(dst + i, m, host_vals + i, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_scal_set(double* S, int s0, double v0, int s1, double v1, int s2, double v2, hipStream_t st) {
    hipLaunchKernelGGL(k_scal_set, dim3(1), dim3(64), 0, st, S, s0, v0, s1, v1, s2, v2);
    return hipGetLastError();
}

hipError_t launch_convert_d2f(const cd* in, cpx<float>* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
hipError_t launch_convert_f2d(const cpx<float>* in, cd* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
hipError_t launch_accum_f(cd* xhi, const cpx<float>* xlo, size_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_accum_lo<float>), dim3(nblk(n)), dim3(256), 0, st, xhi, xlo, n);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pack5(const cd* canon, cpx<R>* half, const Geom& g, int par, int Ns, int refl, hipStream_t st) {
    hipLaunchKernelGGL((k_pack5<R>), dim3(nblk((size_t)g.Vh * 12 * Ns)), dim3(256), 0, st, canon, half, g, par, Ns, refl);
    return hipGetLastError();
}
template hipError_t launch_pack5<double>(const cd*, cd*, const Geom&, int, int, int, hipStream_t);
template hipError_t launch_pack5<float>(const cd*, cpx<float>*, const Geom&, int, int, int, hipStream_t);

template <typename R>
hipError_t launch_unpack5(const cpx<R>* half, cd* canon, const Geom& g, int par, int Ns, int refl, hipStream_t st) {
    hipLaunchKernelGGL((k_unpack5<R>), dim3(nblk((size_t)g.Vh * 12 * Ns)), dim3(256), 0, st, half, canon, g, par, Ns, refl);
    return hipGetLastError();
}
template hipError_t launch_unpack5<double>(const cd*, cd*, const Geom&, int, int, int, hipStream_t);
template hipError_t launch_unpack5<float>(const cpx<float>*, cd*, const Geom&, int, int, int, hipStream_t);

template <typename R>
hipError_t launch_pack_links(const cd* U, cpx<R>* Up, const Geom& g, int par, double tbc, hipStream_t st) {
    hipLaunchKernelGGL((k_pack_links<R>), dim3(nblk((size_t)g.Vh * 36)), dim3(256), 0, st, U, Up, g, par, tbc);
    return hipGetLastError();
}
template hipError_t launch_pack_links<double>(const cd*, cd*, const Geom&, int, double, hipStream_t);
template hipError_t launch_pack_links<float>(const cd*, cpx<float>*, const Geom&, int, double, hipStream_t);

hipError_t launch_source(const cd* phi, cd* half, const Geom& g, int par, int Ns, int chir, const double* coef,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_source, dim3(nblk((size_t)g.Vh * 12 * Ns)), dim3(256), 0, st, phi, half, g, par, Ns, chir, coef);
    return hipGetLastError();
}

hipError_t launch_combine(const cd* phi, const cd* xh, cd* out, const Geom& g, int par, int Ns, int chir, double ck,
                          const double* Om, int accumulate, const Red& red, hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3(nblk((size_t)g.Vh * 12)), dim3(256), 0, st, phi, xh, out, g, par, Ns, chir, ck,
                       Om, accumulate, red);
    finish(red, (unsigned)nblk((size_t)g.Vh * 12), st);
    return hipGetLastError();
}

}  // namespace eofa
