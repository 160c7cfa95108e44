// Stencil Galerkin triple product A^C = R A^F P (Sec. 4.3), one fused kernel
// per (fine pattern, coarsening mask) generated at build time by gen_rap.py
// from the enumerated influence chains.  R = P^T with vertex-centred
// trilinear interpolation; coarse operators are 27-point.  Block systems run
// the same kernel once per block entry (P and R act on each unknown alike).
#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

#include "rap_gen.inc"

hipError_t launch_rap(int pat, int cmask, const Grid& gf, const double* A, long sA, double* Ac, long sAc,
                      hipStream_t st) {
  return rap_dispatch(pat, cmask, gf, A, sA, Ac, sAc, st);
}

int rap_chain_count(int pat, int cmask) { return rap_chain_table(pat, cmask); }

}  // namespace smg
