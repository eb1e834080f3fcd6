// Launchers of the HMC molecular-dynamics kernels (hmc.hip).
#pragma once
#include "eofa_int.h"

namespace eofa {

// Canonical links U[t][z][y][x][mu][3][3] (periodic), momenta and forces P, F[mu][site][8] (site in canonical
// order), T^a = lambda^a / 2.

// partials[block] = sum over the block's sites of sum_{mu < nu} (1 - Re Tr U_mu nu(x) / 3); one block per 256
// sites, red.slot receives the total after launch_finish.
hipError_t launch_plaquette(const cd* U, const Geom& g, const Red& red, hipStream_t st);

// Gauge force of the Wilson plaquette action, dS_g/dw^a = (beta / 3) Im Tr(T^a U A) with A the staple sum:
// written to F (kick == 0) or applied as P -= h F (kick != 0).
hipError_t launch_gauge_force(const cd* U, const Geom& g, double beta, double* F, double* P, double h, int kick,
                              hipStream_t st);

// partials[block] = sum over the block's links of |F| = sqrt(sum_a F^a F^a); one block per 256 links (then
// launch_finish).
hipError_t launch_link_norms(const double* F, size_t nlinks, const Red& red, hipStream_t st);

// P -= h F over n doubles.
hipError_t launch_kick(double* P, const double* F, double h, size_t n, hipStream_t st);

// U_mu(x) <- exp(i h P_mu(x)) U_mu(x).
hipError_t launch_link_update(cd* U, const double* P, double h, const Geom& g, hipStream_t st);

}  // namespace eofa
