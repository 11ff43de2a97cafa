// One instantiation of the factor launcher (tsqr_factor_kernel.hpp), chosen
// by TSQR_INST_T (double or float), TSQR_INST_NP (panels of 16 columns: 1, 2
// or 4) and TSQR_INST_WQ (1: the implicit Q is kept).  The build compiles this
// file once per instantiation; without the macros it compiles to nothing.
#include "tsqr_factor_kernel.hpp"

#if defined(TSQR_INST_T) && defined(TSQR_INST_NP) && defined(TSQR_INST_WQ)
namespace tsqr {
template hipError_t launch_wave<TSQR_INST_T, TSQR_INST_NP, 4, (TSQR_INST_WQ != 0)>(const Geom&, TSQR_INST_T*, int64_t,
                                                                                  const Work&, const TreeArgs&,
                                                                                  hipStream_t);
}  // namespace tsqr
#endif
