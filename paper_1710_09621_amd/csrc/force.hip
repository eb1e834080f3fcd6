// gfx950 kernel of the EOFA fermion force of one chiral action.
//
// S = phi^dag P [1 + c k Om^T H_T^{-1} Om] P phi (Sec. II, Eqs.(m1m2_m1m4), (m1m2_m3m2)) depends on the links only
// through the Wilson hop of D_T.  With x = H_T^{-1} Om P phi and y = gamma_5 R_5 x, the derivative along
// U_mu(x) -> exp(i w^a T^a) U_mu(x) (T^a = lambda^a / 2) is
//   dS/dw^a = -(c k / 2) Im Tr[T^a (U B1 - B2 U^dag)],
//   B1 = sum_s (1 - gamma_mu) x_s(x + mu) (x) y_s(x)^dag,   B2 = sum_s (1 + gamma_mu) x_s(x) (x) y_s(x + mu)^dag,
// spin-traced colour outer products; the packed links carry the t boundary phase, so U is the link the hop uses.
// B1 and B2 are linear in the slice sums, so each slice's share of the 8 components is summed at the end.
#include "force.h"

namespace eofa {

// The upper half of (1 + sg gamma_mu) p in the chiral basis, h = u + sg B_mu d (u, d: spins 0-1 and 2-3).  Since
// B_mu is unitary, the lower half is sg B_mu^dag h, so a spin-traced outer product with (1 + sg gamma_mu) p on one
// side needs only h and the same projection of the other side (see k_force).
__device__ __forceinline__ void half_proj(cd h[6], const cd p[12], int mu, double sg) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cd d0 = p[6 + c], d1 = p[9 + c];
        cd b0, b1;  // B d
        switch (mu) {
        case 0: b0 = cneg(ci(d1)); b1 = cneg(ci(d0)); break;
        case 1: b0 = cneg(d1); b1 = d0; break;
        case 2: b0 = cneg(ci(d0)); b1 = ci(d1); break;
        default: b0 = d0; b1 = d1; break;
        }
        h[c] = {p[c].x + sg * b0.x, p[c].y + sg * b0.y};
        h[3 + c] = {p[3 + c].x + sg * b1.x, p[3 + c].y + sg * b1.y};
    }
}

// Sum of v over the NS lanes of this lane's site group (every lane gets the total).
template <int NS, int OFF = 1>
__device__ __forceinline__ double group_sum(double v, int lane) {
    if constexpr (OFF < NS) {
        v += lane_from<NS, OFF>(v, lane);
        return group_sum<NS, 2 * OFF>(v, lane);
    } else {
        return v;
    }
}

// The hop's lane layout: NS consecutive lanes per site of parity par, lane s of a site handles slice s
// (coalesced column loads).  Each lane forms its slice's share of M = U B1 - B2 U^dag for every mu, turns it
// into the 8 trace components, and the shares are summed over the site's lanes.
template <int NS>
__global__ __launch_bounds__(256) void k_force(const cd* __restrict__ xown, const cd* __restrict__ xoth,
                                               const cd* __restrict__ Uown, Geom g, int par, double kappa,
                                               double* __restrict__ F) {
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63, s = lane & (NS - 1), sb = NS - 1 - s;
    int cb = tid / NS;
    const bool valid = cb < g.Vh;
    if (!valid) cb = g.Vh - 1;  // keep every lane of a group active for the lane exchanges
    int nb[8];
    neighbours(g, cb, par, nb);
    cd x0[12], y0[12];  // x_s(x) and y_s(x) = gamma_5 x_{Ns-1-s}(x)
#pragma unroll
    for (int j = 0; j < 12; j++) {
        x0[j] = xown[((size_t)cb * 12 + j) * NS + s];
        const cd a = xown[((size_t)cb * 12 + j) * NS + sb];
        const double g5 = j < 6 ? 1.0 : -1.0;
        y0[j] = {g5 * a.x, g5 * a.y};
    }
    int lex;
    {
        int xh = cb % g.Lxh, r = cb / g.Lxh;
        const int y = r % g.Ly;
        r /= g.Ly;
        const int z = r % g.Lz, t = r / g.Lz;
        const int x = 2 * xh + ((y + z + t + par) & 1);
        lex = x + g.Lx * (y + g.Ly * (z + g.Lz * t));
    }
    const double r3 = 0.57735026918962576451;  // 1 / sqrt(3)
#pragma unroll 1
    for (int mu = 0; mu < 4; mu++) {
        const int cbf = mu == 0 ? nb[0] : mu == 1 ? nb[2] : mu == 2 ? nb[4] : nb[6];
        // B1 = sum_sp [(1 - gamma) x(x+mu)]_sp (x) y_sp(x)^dag = sum over the two upper spins of a (x) z1^dag with
        // a, z1 the upper halves of (1 - gamma) x(x+mu) and (1 - gamma) y(x); B2 likewise with (1 + gamma)
        cd a[6], z2[6];
        {
            cd xf[12], yf[12];
#pragma unroll
            for (int j = 0; j < 12; j++) {
                xf[j] = xoth[((size_t)cbf * 12 + j) * NS + s];
                const cd b = xoth[((size_t)cbf * 12 + j) * NS + sb];
                const double g5 = j < 6 ? 1.0 : -1.0;
                yf[j] = {g5 * b.x, g5 * b.y};
            }
            half_proj(a, xf, mu, -1.0);
            half_proj(z2, yf, mu, +1.0);
        }
        cd z1[6], c[6];
        half_proj(z1, y0, mu, -1.0);
        half_proj(c, x0, mu, +1.0);
        cd B1[9], B2[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {  // B[i][k] = sum_sp h[sp][i] conj(z[sp][k])
                cd b1 = {0, 0}, b2 = {0, 0};
#pragma unroll
                for (int sp = 0; sp < 2; sp++) {
                    b1 = cjmadd(b1, z1[3 * sp + k], a[3 * sp + i]);
                    b2 = cjmadd(b2, z2[3 * sp + k], c[3 * sp + i]);
                }
                B1[3 * i + k] = b1;
                B2[3 * i + k] = b2;
            }
        cd U[9], M[9];
#pragma unroll
        for (int q = 0; q < 9; q++) U[q] = Uown[((size_t)cb * 4 + mu) * 9 + q];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) {  // M = U B1 - B2 U^dag
                cd m = {0, 0};
#pragma unroll
                for (int l = 0; l < 3; l++) {
                    m = cmadd(m, U[3 * i + l], B1[3 * l + k]);
                    const cd b = B2[3 * i + l], u = U[3 * k + l];  // (U^dag)[l][k] = conj(U[k][l])
                    m.x -= b.x * u.x + b.y * u.y;
                    m.y -= b.y * u.x - b.x * u.y;
                }
                M[3 * i + k] = m;
            }
        // Im Tr[lambda^a M] (Tr[lambda^a M] = sum_ij lambda^a_ij M_ji); Tr[T^a M] = Tr[lambda^a M] / 2
        double im[8];
        im[0] = M[3].y + M[1].y;
        im[1] = -M[3].x + M[1].x;   // Im(-i M10 + i M01)
        im[2] = M[0].y - M[4].y;
        im[3] = M[6].y + M[2].y;
        im[4] = -M[6].x + M[2].x;   // Im(-i M20 + i M02)
        im[5] = M[7].y + M[5].y;
        im[6] = -M[7].x + M[5].x;   // Im(-i M21 + i M12)
        im[7] = r3 * (M[0].y + M[4].y - 2 * M[8].y);
        double* out = F + ((size_t)mu * (2 * (size_t)g.Vh) + lex) * 8;
#pragma unroll
        for (int a = 0; a < 8; a++) {
            const double f = group_sum<NS>(-(kappa / 4) * im[a], lane);
            if (valid && s == 0) out[a] = f;
        }
    }
}

hipError_t launch_force(const cd* xown, const cd* xoth, const cd* Uown, const Geom& g, int par, int Ns, double kappa,
                        double* F, hipStream_t st) {
    const int grid = (int)(((size_t)g.Vh * Ns + 255) / 256);
    switch (Ns) {
    case 4: hipLaunchKernelGGL((k_force<4>), dim3(grid), dim3(256), 0, st, xown, xoth, Uown, g, par, kappa, F); break;
    case 8: hipLaunchKernelGGL((k_force<8>), dim3(grid), dim3(256), 0, st, xown, xoth, Uown, g, par, kappa, F); break;
    case 16: hipLaunchKernelGGL((k_force<16>), dim3(grid), dim3(256), 0, st, xown, xoth, Uown, g, par, kappa, F); break;
    case 32: hipLaunchKernelGGL((k_force<32>), dim3(grid), dim3(256), 0, st, xown, xoth, Uown, g, par, kappa, F); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace eofa
