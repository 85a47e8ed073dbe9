// Mixed-precision multishift CG (FP32/FP16 Krylov bulk, FP64 reliable updates).
#include "mscg.h"

namespace ovl {

size_t mixed_ws_bytes(const Lat &L, int nrhs, int nshift) { return 256; }

int mscg_mixed(const Lat &L, const ovl_gauge *U, double m0, int nshift, const double *shifts, const double *weights,
               Fld b, Fld y, const ovl_solver_params *prm, ovl_solver_stats *stats, char *ws, size_t ws_bytes,
               hipStream_t st)
{
    return OVL_ERR_INVALID;
}

}  // namespace ovl
