// gfx950 kernels of the HMC molecular dynamics (Sec. I; Sec. III): the Wilson plaquette action and its
// force, momentum kicks and the link update.
//
// Sec. III runs the one-flavour HMC with the Wilson plaquette gauge action,
//   S_g = beta sum_{x, mu < nu} (1 - Re Tr U_mu nu(x) / 3),  U_mu nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,
// and Sec. I evolves (U, P) by dU/dtau = i P U, dP^a/dtau = -dH/dw^a, the derivative taken along
// U -> exp(i w^a T^a) U with T^a = lambda^a / 2 (the convention of the fermion force in force.hip).  The link
// U_mu(x) enters S_g as -(beta / 3) Re Tr(U_mu(x) A_mu(x)) with A the sum of its six staples, so
//   dS_g/dw^a = (beta / 3) Im Tr(T^a U A) = (beta / 6) Im Tr(lambda^a U A).
// These kernels work on the canonical (periodic) link array; the fermion boundary phase is applied when the
// links are packed for the hop.  They are memory- and ALU-light next to the fermion forces (one CG solve per
// force), so they use one thread per link and plain 3x3 products.
#include "hmc.h"

namespace eofa {

namespace {

__device__ __forceinline__ void load_su3(const cd* __restrict__ U, int lex, int mu, cd m[9]) {
    const cd* p = U + ((size_t)lex * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; k++) m[k] = p[k];
}

// c = a b
__device__ __forceinline__ void mul_nn(const cd a[9], const cd b[9], cd c[9]) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cd s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) s = cmadd(s, a[3 * i + k], b[3 * k + j]);
            c[3 * i + j] = s;
        }
}

// c = a b^dag
__device__ __forceinline__ void mul_nd(const cd a[9], const cd b[9], cd c[9]) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cd s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) s = cjmadd(s, b[3 * j + k], a[3 * i + k]);  // a_ik conj(b_jk)
            c[3 * i + j] = s;
        }
}

// c = a^dag b
__device__ __forceinline__ void mul_dn(const cd a[9], const cd b[9], cd c[9]) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cd s = {0, 0};
#pragma unroll
            for (int k = 0; k < 3; k++) s = cjmadd(s, a[3 * k + i], b[3 * k + j]);  // conj(a_ki) b_kj
            c[3 * i + j] = s;
        }
}

// Canonical index of the site lex shifted by d (+1 or -1) in direction mu, periodic.
__device__ __forceinline__ int lex_step(const Geom& g, int lex, int mu, int d) {
    int x = lex % g.Lx, r = lex / g.Lx;
    int y = r % g.Ly;
    r /= g.Ly;
    int z = r % g.Lz, t = r / g.Lz;
    if (mu == 0) x = (x + d + g.Lx) % g.Lx;
    else if (mu == 1) y = (y + d + g.Ly) % g.Ly;
    else if (mu == 2) z = (z + d + g.Lz) % g.Lz;
    else t = (t + d + g.Lt) % g.Lt;
    return x + g.Lx * (y + g.Ly * (z + g.Lz * t));
}

// Im Tr(lambda^a M), a = 1..8 (Tr(lambda M) = sum_ij lambda_ij M_ji).
__device__ __forceinline__ void im_tr_lambda(const cd M[9], double o[8]) {
    const double r3 = 0.57735026918962576451;  // 1 / sqrt(3)
    o[0] = M[3].y + M[1].y;
    o[1] = M[1].x - M[3].x;
    o[2] = M[0].y - M[4].y;
    o[3] = M[6].y + M[2].y;
    o[4] = M[2].x - M[6].x;
    o[5] = M[7].y + M[5].y;
    o[6] = M[5].x - M[7].x;
    o[7] = r3 * (M[0].y + M[4].y - 2 * M[8].y);
}

// X = i sum_a p^a T^a (anti-Hermitian, traceless), from the 8 real components.
__device__ __forceinline__ void i_algebra(const double p[8], double h, cd X[9]) {
    const double r3 = 0.57735026918962576451;
    // Q = sum_a p^a lambda^a / 2 (Hermitian)
    cd Q[9];
    Q[0] = {0.5 * (p[2] + r3 * p[7]), 0};
    Q[4] = {0.5 * (-p[2] + r3 * p[7]), 0};
    Q[8] = {-r3 * p[7], 0};
    Q[1] = {0.5 * p[0], -0.5 * p[1]};
    Q[3] = {0.5 * p[0], 0.5 * p[1]};
    Q[2] = {0.5 * p[3], -0.5 * p[4]};
    Q[6] = {0.5 * p[3], 0.5 * p[4]};
    Q[5] = {0.5 * p[5], -0.5 * p[6]};
    Q[7] = {0.5 * p[5], 0.5 * p[6]};
#pragma unroll
    for (int k = 0; k < 9; k++) X[k] = {-h * Q[k].y, h * Q[k].x};  // i h Q
}

// exp(X) by scaling and squaring: Y = X / 2^s with |Y|_F <= 1/2, the Taylor polynomial of degree 18 in
// Horner form (remainder at most |Y|^19 / 19! < 2e-23), then s squarings.
__device__ __forceinline__ void su3_exp(const cd X[9], cd E[9]) {
    double n2 = 0;
#pragma unroll
    for (int k = 0; k < 9; k++) n2 += X[k].x * X[k].x + X[k].y * X[k].y;
    int s = 0;
    double sc = 1.0;
    while (n2 > 0.25 && s < 64) {  // |X / 2^s|_F^2 <= 1/4
        n2 *= 0.25;
        sc *= 0.5;
        s++;
    }
    cd Y[9];
#pragma unroll
    for (int k = 0; k < 9; k++) Y[k] = {sc * X[k].x, sc * X[k].y};
    // E = I + Y/1 (I + Y/2 (I + ... (I + Y/18)))
    cd T[9];
#pragma unroll
    for (int k = 0; k < 9; k++) E[k] = {(k % 4 == 0) ? 1.0 : 0.0, 0.0};
#pragma unroll 1
    for (int n = 18; n >= 1; n--) {
        const double inv = 1.0 / n;
        mul_nn(Y, E, T);
#pragma unroll
        for (int k = 0; k < 9; k++) E[k] = {((k % 4 == 0) ? 1.0 : 0.0) + inv * T[k].x, inv * T[k].y};
    }
#pragma unroll 1
    for (int i = 0; i < s; i++) {
        mul_nn(E, E, T);
#pragma unroll
        for (int k = 0; k < 9; k++) E[k] = T[k];
    }
}

__global__ __launch_bounds__(256) void k_plaquette(const cd* __restrict__ U, Geom g, Red red) {
    __shared__ double lds[4];
    const int V = 2 * g.Vh;
    const int lex = blockIdx.x * 256 + threadIdx.x;
    double v = 0;
    if (lex < V) {
#pragma unroll 1
        for (int mu = 0; mu < 3; mu++) {
            cd Um[9], A[9], B[9], W[9];
            load_su3(U, lex, mu, Um);
            const int xm = lex_step(g, lex, mu, +1);
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; nu++) {
                const int xn = lex_step(g, lex, nu, +1);
                load_su3(U, xm, nu, W);
                mul_nn(Um, W, A);  // U_mu(x) U_nu(x + mu)
                cd Un[9];
                load_su3(U, lex, nu, Un);
                load_su3(U, xn, mu, W);
                mul_nn(Un, W, B);  // U_nu(x) U_mu(x + nu)
                double tr = 0;     // Re Tr(A B^dag) = sum_ij Re(A_ij conj(B_ij))
#pragma unroll
                for (int k = 0; k < 9; k++) tr += A[k].x * B[k].x + A[k].y * B[k].y;
                v += 1.0 - tr / 3.0;
            }
        }
    }
    finish_sum(red, block_sum256(v, lds));
}

// Four lanes per link (a quad of consecutive lanes): lane nu forms the two staples of the plane (mu, nu) (none when
// nu == mu), the quad sums them, and every lane forms M = U A and writes two of the eight components.
__global__ __launch_bounds__(256) void k_gauge_force(const cd* __restrict__ U, Geom g, double beta,
                                                     double* __restrict__ F, double* __restrict__ P, double h,
                                                     int kick) {
    const int V = 2 * g.Vh;
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int link = tid >> 2, nu = tid & 3;
    const bool valid = link < 4 * V;  // whole quads are in or out: 4 V links, 256-lane blocks
    const int mu = valid ? link / V : 0, lex = valid ? link - mu * V : 0;
    cd A[9];
#pragma unroll
    for (int k = 0; k < 9; k++) A[k] = {0, 0};
    if (valid && nu != mu) {
        cd a[9], b[9], c[9], t[9];
        const int xm = lex_step(g, lex, mu, +1);
        // upper staple U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag
        load_su3(U, xm, nu, a);
        load_su3(U, lex_step(g, lex, nu, +1), mu, b);
        load_su3(U, lex, nu, c);
        mul_nd(a, b, t);
        mul_nd(t, c, A);
        // lower staple U_nu(x + mu - nu)^dag U_mu(x - nu)^dag U_nu(x - nu) = (U_mu(x - nu) U_nu(x + mu - nu))^dag U_nu(x - nu)
        const int xd = lex_step(g, lex, nu, -1);
        load_su3(U, lex_step(g, xm, nu, -1), nu, a);
        load_su3(U, xd, mu, b);
        load_su3(U, xd, nu, c);
        mul_nn(b, a, t);
        mul_dn(t, c, a);
#pragma unroll
        for (int k = 0; k < 9; k++) A[k] = cadd(A[k], a[k]);
    }
    // quad sum ((A_0 + A_1) + (A_2 + A_3)), the same order in every lane
#pragma unroll
    for (int k = 0; k < 9; k++) {
        A[k].x += __shfl_xor(A[k].x, 1, 4);
        A[k].y += __shfl_xor(A[k].y, 1, 4);
        A[k].x += __shfl_xor(A[k].x, 2, 4);
        A[k].y += __shfl_xor(A[k].y, 2, 4);
    }
    if (!valid) return;
    cd Um[9], M[9];
    load_su3(U, lex, mu, Um);
    mul_nn(Um, A, M);
    double o[8];
    im_tr_lambda(M, o);
    const double f = beta / 6.0;
    // components 2 nu and 2 nu + 1 (selects: a runtime index would move o[] to scratch memory)
    const double v0 = f * (nu == 0 ? o[0] : nu == 1 ? o[2] : nu == 2 ? o[4] : o[6]);
    const double v1 = f * (nu == 0 ? o[1] : nu == 1 ? o[3] : nu == 2 ? o[5] : o[7]);
    double* q = (kick ? P : F) + (size_t)link * 8 + 2 * nu;
    if (kick) {
        q[0] -= h * v0;
        q[1] -= h * v1;
    } else {
        q[0] = v0;
        q[1] = v1;
    }
}

// partials of sum over links of |F| = sqrt(sum_a F^a F^a) (one thread per link)
__global__ __launch_bounds__(256) void k_link_norms(const double* __restrict__ F, size_t nlinks, Red red) {
    __shared__ double lds[4];
    const size_t l = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0;
    if (l < nlinks) {
        const double* f = F + l * 8;
#pragma unroll
        for (int a = 0; a < 8; a++) v = fma(f[a], f[a], v);
        v = sqrt(v);
    }
    finish_sum(red, block_sum256(v, lds));
}

__global__ __launch_bounds__(256) void k_kick(double* __restrict__ P, const double* __restrict__ F, double h, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) P[i] -= h * F[i];
}

__global__ __launch_bounds__(256) void k_link_update(cd* __restrict__ U, const double* __restrict__ P, double h, Geom g) {
    const int V = 2 * g.Vh;
    const int tid = blockIdx.x * 256 + threadIdx.x;
    if (tid >= 4 * V) return;
    const int mu = tid / V, lex = tid - mu * V;
    double p[8];
#pragma unroll
    for (int a = 0; a < 8; a++) p[a] = P[(size_t)tid * 8 + a];
    cd X[9], E[9], Uo[9], Un[9];
    i_algebra(p, h, X);
    su3_exp(X, E);
    load_su3(U, lex, mu, Uo);
    mul_nn(E, Uo, Un);
    cd* d = U + ((size_t)lex * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; k++) d[k] = Un[k];
}

}  // namespace

hipError_t launch_plaquette(const cd* U, const Geom& g, const Red& red, hipStream_t st) {
    const int V = 2 * g.Vh;
    hipLaunchKernelGGL(k_plaquette, dim3((V + 255) / 256), dim3(256), 0, st, U, g, red);
    return hipGetLastError();
}

hipError_t launch_gauge_force(const cd* U, const Geom& g, double beta, double* F, double* P, double h, int kick,
                              hipStream_t st) {
    const long n = 4 * 8 * (long)g.Vh;  // four lanes per link, 4 V links
    if (n > (1l << 31) - 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gauge_force, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U, g, beta, F, P, h, kick);
    return hipGetLastError();
}

hipError_t launch_link_norms(const double* F, size_t nlinks, const Red& red, hipStream_t st) {
    const size_t b = (nlinks + 255) / 256;
    hipLaunchKernelGGL(k_link_norms, dim3((unsigned)b), dim3(256), 0, st, F, nlinks, red);
    return hipGetLastError();
}

hipError_t launch_kick(double* P, const double* F, double h, size_t n, hipStream_t st) {
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_kick, dim3((unsigned)b), dim3(256), 0, st, P, F, h, n);
    return hipGetLastError();
}

hipError_t launch_link_update(cd* U, const double* P, double h, const Geom& g, hipStream_t st) {
    const int n = 8 * g.Vh;
    hipLaunchKernelGGL(k_link_update, dim3((n + 255) / 256), dim3(256), 0, st, U, P, h, g);
    return hipGetLastError();
}

}  // namespace eofa
