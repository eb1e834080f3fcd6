// Launcher of the EOFA fermion-force kernel (force.hip).
#pragma once
#include "eofa_int.h"

namespace eofa {

// F[mu][lex][a] for the links U_mu(x) of the sites of parity par: xown / xoth = the 5D solution x on
// parity par / 1 - par (internal half layout), Uown = packed links of parity par, kappa = c k.
hipError_t launch_force(const cd* xown, const cd* xoth, const cd* Uown, const Geom& g, int par, int Ns, double kappa,
                        double* F, hipStream_t st);

}  // namespace eofa
